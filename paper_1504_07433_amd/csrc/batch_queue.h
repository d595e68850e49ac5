// batch_queue.h -- the work list of the persistent batch kernel: tiles (a
// light curve's run of exposures), their order, the per-light-curve tile
// lists of the likelihood reduction, and the pop protocol of the tile queue.
// Plain host/device code without HIP calls, so that the host tests build it
// with the system compiler.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>
#include <vector>

namespace pt {

// The tile queue is split into kQueues sub-queues (tile q + i kQueues is the
// i-th tile of sub-queue q), each with its own counter on its own 128-byte
// line: one counter serialises its atomics at the memory side, and the pops
// of all waves of the GPU otherwise meet on it.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;   // unsigned ints between counters
constexpr int kWaveLanes = 64;

// One unit of the persistent queue: exposures e0 .. e0+ne-1 of light curve
// lc, in every band of it (bands = 0) or in bands lo .. lo+cnt-1 counted from
// the light curve's first (bands = lo | cnt << 16, cnt >= 1).
struct TileDesc {
  int32_t lc;
  int32_t e0;
  int32_t ne;
  int32_t bands;
};

constexpr int kTileBandsMax = 0x7fff;   // bands of a light curve whose tiles may be split by band
constexpr int kTileSplitMinBands = 8;   // bands per piece of a split tile, at least
constexpr int kTileSplitMaxPieces = 4;  // band pieces of one tile, at most
constexpr int kTileTailWaves = 1;       // tiles split at the end of the order, per wave of the grid

__host__ __device__ __forceinline__ int32_t tile_bands(int lo, int cnt) { return lo | (cnt << 16); }

// The next tile for a wave.  `pop(q)` returns the old value of sub-queue q's
// counter and increments it (an atomic on the GPU, wave-uniform).  A wave
// starts on sub-queue q0 and moves on when the one it is on runs dry; since
// counters only grow, a sub-queue that ran dry stays dry, so after kQueues
// dry pops every sub-queue is exhausted and the function returns false.
// Between two calls the caller keeps q and dry.
template <class Pop>
__host__ __device__ __forceinline__ bool next_tile(int& q, int& dry, int64_t n_tiles, Pop pop, uint32_t* tile) {
  for (;;) {
    const unsigned int pos = pop(q);
    const uint64_t t = (uint64_t)pos * kQueues + (uint64_t)q;
    if (t < (uint64_t)n_tiles) {
      *tile = (uint32_t)t;
      return true;
    }
    if (++dry == kQueues) return false;
    q = q + 1 == kQueues ? 0 : q + 1;
  }
}

// Work estimate of a tile: wave iterations x subsamples x (bands + the orbit).
inline double tile_work(int ne, int nss, int nb) {
  return double((ne + kWaveLanes - 1) / kWaveLanes) * nss * (nb + 1.0);
}

// Tiles of a batch, longest first (ties in light-curve and exposure order, so
// neighbouring tiles share cache lines), and per light curve the list of its
// tile indices (CSR: lc_off[n_lc + 1], lc_tiles[n_tiles], in tile order).
// Light curves without bands or exposures get no tile.
//
// The last `tail` tiles of that order, of light curves with 2
// kTileSplitMinBands bands or more, are split into up to kTileSplitMaxPieces
// runs of their bands.  The queue hands out tiles in order, so the grid's
// last tiles are short and its waves finish closer together; each piece
// solves the orbit of its exposures again (the bands of a piece share it).
// Tiles are not split by exposures: on batches of one band that cost more
// than the shorter tail saved.
struct TilePlan {
  std::vector<TileDesc> tiles;
  std::vector<int32_t> lc_off, lc_tiles;
};

inline void make_tile_plan(int32_t n_lc, const int64_t* t_count, const int32_t* nss, const int32_t* band_off,
                           int tile_e, int64_t tail, TilePlan* out) {
  struct W {
    double work;
    TileDesc t;
  };
  auto by_work = [](const W& a, const W& b) { return a.work > b.work; };
  std::vector<W> v;
  for (int32_t lc = 0; lc < n_lc; ++lc) {
    const int nb = band_off[lc + 1] - band_off[lc];
    if (nb == 0) continue;
    for (int64_t e0 = 0; e0 < t_count[lc]; e0 += tile_e) {
      const int ne = (int)std::min<int64_t>(tile_e, t_count[lc] - e0);
      v.push_back({tile_work(ne, nss[lc], nb), TileDesc{lc, (int32_t)e0, ne, 0}});
    }
  }
  std::stable_sort(v.begin(), v.end(), by_work);
  const size_t head = v.size() - (tail > 0 ? std::min<size_t>((size_t)tail, v.size()) : 0);
  std::vector<W> pieces;
  for (size_t j = head; j < v.size(); ++j) {
    const TileDesc& t = v[j].t;
    const int nb = band_off[t.lc + 1] - band_off[t.lc];
    const int np = nb <= kTileBandsMax ? std::min(kTileSplitMaxPieces, nb / kTileSplitMinBands) : 1;
    if (np < 2) {
      pieces.push_back(v[j]);
      continue;
    }
    for (int p = 0; p < np; ++p) {
      const int lo = (int)((int64_t)nb * p / np), hi = (int)((int64_t)nb * (p + 1) / np);
      pieces.push_back({tile_work(t.ne, nss[t.lc], hi - lo), TileDesc{t.lc, t.e0, t.ne, tile_bands(lo, hi - lo)}});
    }
  }
  std::stable_sort(pieces.begin(), pieces.end(), by_work);
  out->tiles.resize(head + pieces.size());
  for (size_t i = 0; i < head; ++i) out->tiles[i] = v[i].t;
  for (size_t i = 0; i < pieces.size(); ++i) out->tiles[head + i] = pieces[i].t;
  out->lc_off.assign((size_t)n_lc + 1, 0);
  out->lc_tiles.resize(out->tiles.size());
  for (const TileDesc& t : out->tiles) out->lc_off[t.lc + 1]++;
  for (int32_t i = 0; i < n_lc; ++i) out->lc_off[i + 1] += out->lc_off[i];
  std::vector<int32_t> fill(out->lc_off.begin(), out->lc_off.end() - 1);
  for (size_t j = 0; j < out->tiles.size(); ++j) out->lc_tiles[fill[out->tiles[j].lc]++] = (int32_t)j;
}

}  // namespace pt
