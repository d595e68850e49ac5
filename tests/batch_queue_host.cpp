// Host build of the batch kernel's work list (paper_1504_07433_amd/csrc/
// batch_queue.h) for the CPU tests: the tile plan of a batch shape, the
// persistent queue's pops by many waves in a random interleaving (the same
// next_tile the kernel runs, with a plain counter in place of the atomic), the
// per-tile partial sums of the likelihood and their per-light-curve reduction
// in tile-list order.
#include <algorithm>
#include <cstring>
#include <random>

#include "../paper_1504_07433_amd/csrc/batch_queue.h"

extern "C" {

// Returns 0 when every check holds, else a code naming the first failure:
//   1 a tile index out of range, 2 a tile taken twice, 3 a tile never taken,
//   4 a wave popped more than (its tiles + kQueues) times, 5 a light curve's
//   tile list holds another light curve's tile or misses one of its own,
//   6 a reduced sum differs from the direct sum over the light curve's tiles,
//   7 a tile's exposures or bands leave its light curve, 8 tiles not in work
//   order (the whole tiles, then the pieces of the split tail, each longest
//   first), 9 an (exposure, band) element of a light curve in no tile or in
//   two, 10 a tail tile of a light curve with enough bands left whole, split
//   into too few bands, or a tile before the tail split.
// tail: tiles split at the end of the order (make_tile_plan).
// stats[0] = tiles, stats[1] = pops, stats[2] = largest pops of one wave,
// stats[3] = tiles that are pieces of the split tail.
int queue_check(int32_t n_lc, const int64_t* t_count, const int32_t* nss, const int32_t* band_off, int tile_e,
                int64_t tail, int n_workgroups, int waves_per_group, unsigned seed, int64_t* stats) {
  pt::TilePlan tp;
  pt::make_tile_plan(n_lc, t_count, nss, band_off, tile_e, tail, &tp);
  const int64_t n_tiles = (int64_t)tp.tiles.size();
  auto nb_of = [&](const pt::TileDesc& t) {
    return t.bands ? t.bands >> 16 : band_off[t.lc + 1] - band_off[t.lc];
  };
  // the whole tiles come first: those of the plan without a tail, less the
  // `tail` it splits
  pt::TilePlan whole;
  pt::make_tile_plan(n_lc, t_count, nss, band_off, tile_e, 0, &whole);
  const int64_t n_whole = (int64_t)whole.tiles.size();
  const int64_t n_split = tail > 0 ? std::min<int64_t>(tail, n_whole) : 0;
  const int64_t head = n_whole - n_split;
  std::vector<std::vector<uint8_t>> cover(n_lc);
  for (int32_t lc = 0; lc < n_lc; ++lc)
    cover[lc].assign((size_t)t_count[lc] * (size_t)(band_off[lc + 1] - band_off[lc]), 0);
  for (int64_t j = 0; j < n_tiles; ++j) {
    const pt::TileDesc& t = tp.tiles[j];
    if (t.lc < 0 || t.lc >= n_lc || t.e0 < 0 || t.ne < 1 || t.e0 + t.ne > t_count[t.lc]) return 7;
    const int nb = band_off[t.lc + 1] - band_off[t.lc];
    const int lo = t.bands & 0xffff, cnt = nb_of(t);
    if (cnt < 1 || lo + cnt > nb) return 7;
    for (int e = t.e0; e < t.e0 + t.ne; ++e)
      for (int b = lo; b < lo + cnt; ++b)
        if (cover[t.lc][(size_t)b * t_count[t.lc] + e]++) return 9;
    if (j >= head) {
      if (t.bands && cnt < pt::kTileSplitMinBands) return 10;
      if (!t.bands && nb >= 2 * pt::kTileSplitMinBands && nb <= pt::kTileBandsMax) return 10;
    } else if (t.bands) {
      return 10;
    }
    if (j > 0 && j != head) {
      const pt::TileDesc& u = tp.tiles[j - 1];
      const double wu = pt::tile_work(u.ne, nss[u.lc], nb_of(u));
      const double wt = pt::tile_work(t.ne, nss[t.lc], cnt);
      if (wt > wu) return 8;
    }
  }
  for (int32_t lc = 0; lc < n_lc; ++lc)
    for (uint8_t c : cover[lc])
      if (c != 1) return 9;
  // waves of the persistent grid: wave w belongs to workgroup w / waves_per_group
  const int n_waves = n_workgroups * waves_per_group;
  std::vector<unsigned int> counter(pt::kQueues, 0u);
  std::vector<int> q(n_waves), dry(n_waves, 0), done(n_waves, 0);
  std::vector<int64_t> pops(n_waves, 0), taken_by(n_tiles, -1);
  std::vector<int64_t> mine(n_waves, 0);
  for (int w = 0; w < n_waves; ++w) q[w] = (w / waves_per_group) % pt::kQueues;
  std::vector<double> partial(n_tiles, 0.0);
  std::mt19937 rng(seed);
  std::vector<int> live(n_waves);
  for (int w = 0; w < n_waves; ++w) live[w] = w;
  int64_t total_pops = 0;
  while (!live.empty()) {
    const size_t pick = rng() % live.size();
    const int w = live[pick];
    auto pop = [&](int qq) {
      ++pops[w];
      ++total_pops;
      return counter[qq]++;
    };
    uint32_t tid = 0;
    if (pt::next_tile(q[w], dry[w], n_tiles, pop, &tid)) {
      if ((int64_t)tid >= n_tiles) return 1;
      if (taken_by[tid] >= 0) return 2;
      taken_by[tid] = w;
      ++mine[w];
      partial[tid] = 1.0 + 0.001 * tid;   // the tile's partial sum
    } else {
      live[pick] = live.back();
      live.pop_back();
    }
  }
  int64_t max_pops = 0;
  for (int64_t j = 0; j < n_tiles; ++j)
    if (taken_by[j] < 0) return 3;
  for (int w = 0; w < n_waves; ++w) {
    if (pops[w] > mine[w] + pt::kQueues) return 4;
    max_pops = std::max(max_pops, pops[w]);
  }
  // per-light-curve lists and the reduction in list order
  std::vector<int> seen(n_tiles, 0);
  for (int32_t lc = 0; lc < n_lc; ++lc) {
    double s = 0.0, direct = 0.0;
    for (int32_t j = tp.lc_off[lc]; j < tp.lc_off[lc + 1]; ++j) {
      const int32_t t = tp.lc_tiles[j];
      if (t < 0 || t >= n_tiles || tp.tiles[t].lc != lc || seen[t]++) return 5;
      s += partial[t];
    }
    for (int64_t t = 0; t < n_tiles; ++t)
      if (tp.tiles[t].lc == lc) direct += partial[t];
    if (std::abs(s - direct) > 1e-9 * (1.0 + std::abs(direct))) return 6;
  }
  for (int64_t t = 0; t < n_tiles; ++t)
    if (!seen[t]) return 5;
  stats[0] = n_tiles;
  stats[1] = total_pops;
  stats[2] = max_pops;
  stats[3] = n_tiles - head;
  return 0;
}

}  // extern "C"
