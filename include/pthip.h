/* pthip.h -- C ABI of the MI355X (gfx950) transit-model library libpthip.so.
 *
 * The forward transit model of PyTransit (Parviainen 2015): the orbit
 * (Kepler's equation by Newton's method, sky-projected distance z; Sect. 1),
 * the quadratic Mandel & Agol (2002) model factored so that the limb
 * darkening enters only at the end (Sect. 2.2, eq. ma_model), the Gimenez
 * (2006) Jacobi-series model with the general limb-darkening law (Sect. 2.1,
 * eqs. gimenez_flux .. gimemez_a, ld_general), many passbands at once
 * (Sects. 2.1.3, 2.2.2) and supersampled exposures (Sect. 3.2).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    HOST; the library never frees or retains them beyond the call.
 *  - Every call validates its arguments on the host before any launch (an
 *    error never leaves a partial launch), enqueues its work on `stream`
 *    (a hipStream_t passed as void*, NULL = the default stream) and returns
 *    without synchronising.  Results are ready once the stream is.
 *  - On failure the return value is not PT_OK and pt_last_error() gives a
 *    message for the calling thread; nothing is enqueued.
 *  - Kernels never trap.  Non-physical values that cannot be checked on the
 *    host (device-resident parameters: e >= 1, aR <= 0, P <= 0, b < 0 or an
 *    inclination with cos i > 1) give NaN flux for the light curves they
 *    belong to, and a radius ratio that is not positive and finite, or
 *    limb-darkening coefficients whose flux weights are not finite, give NaN
 *    flux for their passband; NaN inputs give NaN outputs.
 *  - z < 0 marks the planet behind the star; its flux is 1.
 *  - Calls on different streams may run concurrently; the library's own
 *    caches are guarded by a mutex.
 */
#ifndef PTHIP_H
#define PTHIP_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PT_OK = 0,
  PT_ERR_ARG = 1,          /* invalid argument (message names it)          */
  PT_ERR_HIP = 2,          /* a HIP runtime call failed                    */
  PT_ERR_NOMEM = 3,        /* device or host allocation failed             */
  PT_ERR_UNSUPPORTED = 4   /* valid request this library does not provide  */
} pt_status;

typedef enum {
  PT_PREC_FP64 = 0,        /* double throughout                                     */
  PT_PREC_FP32 = 1,        /* float orbit and limb terms; the Mandel-Agol elliptic   */
                           /* combination in double FMAs seeded by float hardware    */
                           /* reciprocals; exact double within 1e-6 of z = k, 1 - k  */
                           /* and for k > 1/2; Gimenez series in float               */
  PT_PREC_SURROGATE = 2    /* PT_PREC_FP32 with the Mandel-Agol functions from the   */
                           /* learned network where it is valid (pt_surrogate_set)   */
} pt_prec;

typedef enum {
  PT_MODEL_MA_QUAD = 0,    /* quadratic Mandel & Agol; u rows are (u1, u2)                 */
  PT_MODEL_GIMENEZ = 1,    /* Gimenez; u rows are the general-law u_1..u_nldc              */
  PT_MODEL_MA_INTERP = 2,  /* quadratic Mandel & Agol with lambda_e, lambda_d, eta_d from  */
                           /* bilinear tables (Sect. 2.2.3; pt_ma_table_set); float path  */
  PT_MODEL_MA_KHAT = 3,    /* quadratic Mandel & Agol evaluated at each light curve's mean */
                           /* radius ratio khat, depth scaled by k_i^2/khat^2 per band     */
                           /* (Sect. 3.5; an approximation); float path                    */
  PT_MODEL_GIMENEZ_ZINTERP = 4  /* Gimenez flux interpolated linearly in z between nodes  */
                           /* tabulated per band (Sect. 3.3; pt_gimenez_zgrid_set); float */
} pt_model;

/* Library version, e.g. "pthip 1.0 gfx950". */
const char* pt_version(void);

/* Message for the last failed call on this thread ("" if none). */
const char* pt_last_error(void);

/* Frees library-owned caches (coefficient tables, batch plans, graphs,
 * surrogate weights) on every device.  Not safe while calls are in flight. */
void pt_release(void);

/* Compute units of the current device (for launch sizing); <= 0 on error. */
int pt_device_cu_count(void);

/* Signed projected distance z(t) (Sect. 1; orbit by Newton's method).
 *   t[n]   exposure times (days), device, double
 *   t0     time of inferior conjunction; P period (days, > 0); aR = a/R* (> 0)
 *   b      transit impact parameter a cos i (1-e^2)/(1+e sin w) / R* (>= 0)
 *   e      eccentricity in [0, 1); w argument of periastron (radians)
 *   prec   PT_PREC_FP64 or PT_PREC_FP32 (conjunction-frame float solve)
 *   z[n]   output, device, double; negative = behind the star
 * Errors: PT_ERR_ARG for n < 0, NULL pointers with n > 0, non-physical
 * parameters (named in the message). */
pt_status pt_orbit_z(const double* t, int64_t n, double t0, double P, double aR, double b,
                     double e, double w, pt_prec prec, double* z, void* stream);

/* Quadratic Mandel-Agol flux for one radius ratio k and nb passbands
 * (Sect. 2.2, eq. ma_model; passbands share the k,z-dependent functions,
 * Sect. 2.2.2).
 *   z[n]        projected distances, device, double
 *   k           radius ratio (> 0)
 *   u[nb][2]    quadratic coefficients (u1, u2) per band, device, double;
 *               1 - u1/3 - u2/6 must be non-zero
 *   prec        PT_PREC_FP64 or PT_PREC_FP32
 *   flux[nb][n] output, device, double (band-major)
 * Errors: PT_ERR_ARG for n < 0, nb < 1, k <= 0, NULL pointers. */
pt_status pt_ma_quad(const double* z, int64_t n, double k, const double* u, int32_t nb,
                     pt_prec prec, double* flux, void* stream);

/* Gimenez flux for one radius ratio and nb passbands of the general law
 * I(mu)/I(1) = 1 - sum_n u_n (1 - mu^n) (Sect. 2.1, eqs. gimenez_alpha,
 * gimenez, ld_general; C_n of Sect. 2.1.3).  The series is truncated to npol
 * Jacobi terms (j = 0 .. npol-1).  A quadratic law (a, b) is the general law
 * u_1 = a + 2b, u_2 = -b (Sect. 2.1.2).
 *   z[n], k, flux[nb][n] as for pt_ma_quad
 *   u[nb][nldc] general-law coefficients, device, double; 1 <= nldc <= 4
 *   npol        1 .. 512
 * Errors: PT_ERR_ARG for out-of-range sizes or NULL pointers. */
pt_status pt_gimenez(const double* z, int64_t n, double k, const double* u, int32_t nldc,
                     int32_t nb, int32_t npol, pt_prec prec, double* flux, void* stream);

/* Builds the interpolation tables of PT_MODEL_MA_INTERP (Sect. 2.2.3): the
 * three functions lambda_e, lambda_d + 2/3 Theta(k-z), eta_d from the exact
 * double path on a uniform grid of nk radius ratios in [k_lo, k_hi] and nz
 * distances in [0, 1 + k_hi]; evaluation is bilinear in (k, z).  Radius
 * ratios outside [k_lo, k_hi] use the exact float path.  The table is
 * library-owned (one per device) and ready when the call returns.  Each
 * pt_lc_batch call with PT_MODEL_MA_INTERP also keeps 2 nz floats per
 * passband (the band's weighted sum at the z nodes, as pairs of neighbours)
 * in its cached batch plan when these take at most 64 MB; larger batches
 * interpolate the shared table directly (same values up to rounding).
 * Errors: PT_ERR_ARG unless 0 < k_lo < k_hi, nk >= 2, nz >= 2,
 * nk * nz <= 2^24. */
pt_status pt_ma_table_set(double k_lo, double k_hi, int32_t nk, int32_t nz, void* stream);

/* Node counts of PT_MODEL_GIMENEZ_ZINTERP (Sect. 3.3): n_in nodes on
 * [0, 1-k] and n_limb nodes on [1-k, 1+k] per band (defaults 50 and 50).
 * Applies to later calls.  Errors: PT_ERR_ARG unless 2 <= n <= 65536. */
pt_status pt_gimenez_zgrid_set(int32_t n_in, int32_t n_limb);

/* A ragged batch of light curves: each has its own orbit, exposure times,
 * exposure time and supersampling factor, and its own passbands, each with
 * its own radius ratio and limb darkening (Sects. 1, 2.1.3, 2.2.2, 3.2).
 * Shape arrays are HOST arrays: they are validated and copied into a cached
 * plan (keyed by their contents) on first use.  Values are DEVICE arrays. */
typedef struct {
  int32_t n_lc;              /* light curves (>= 0)                                    */
  int32_t nldc;              /* coefficients per band: 2 for PT_MODEL_MA_QUAD,          */
                             /* 1..4 for PT_MODEL_GIMENEZ                               */
  int64_t n_t;               /* length of the time pool t                              */
  int64_t n_flux;            /* length of the output array                             */
  /* HOST shape arrays */
  const int64_t* t_start;    /* [n_lc] first exposure of light curve i in t            */
  const int64_t* t_count;    /* [n_lc] exposures of light curve i (>= 0)               */
  const int32_t* nss;        /* [n_lc] subsamples per exposure (>= 1)                  */
  const int32_t* band_off;   /* [n_lc+1] bands of i are band_off[i] .. band_off[i+1]-1 */
  const int64_t* flux_off;   /* [n_lc] start of light curve i's output block,          */
                             /* laid out [n_band_i][t_count_i]; blocks must not overlap */
  /* DEVICE value arrays (double) */
  const double* t;           /* [n_t] exposure mid-times (days)                        */
  const double* t0;          /* [n_lc] time of inferior conjunction                    */
  const double* P;           /* [n_lc] period                                          */
  const double* aR;          /* [n_lc] a / R*                                          */
  const double* b;           /* [n_lc] transit impact parameter                        */
  const double* e;           /* [n_lc] eccentricity                                    */
  const double* w;           /* [n_lc] argument of periastron (radians)                */
  const double* t_exp;       /* [n_lc] exposure time (days); subsample s of n sits at  */
                             /* t + t_exp ((s + 1/2)/n - 1/2)                           */
  const double* k;           /* [band_off[n_lc]] radius ratio per band (> 0)            */
  const double* u;           /* [band_off[n_lc]][nldc] limb darkening per band          */
} pt_batch;

/* Supersampled flux of a ragged batch in one persistent fused orbit+flux
 * launch (replayed from a hipGraph after the first call with a given shape).
 * Each output point is the mean over the exposure's subsamples (Sect. 3.2).
 * The float precisions solve Kepler's equation once per exposure and take
 * the subsamples' sky positions from power series about its centre where a
 * rigorous truncation bound keeps z within 3e-8 (4..16 subsamples; otherwise
 * one solve per subsample); PT_PREC_FP64 solves per subsample.  A light curve
 * with non-physical orbit parameters, or a band with a radius ratio that is
 * not positive and finite or with non-finite limb-darkening weights, gives
 * NaN in every affected output point.
 *   flux    output [n_flux], device: float for PT_PREC_FP32/PT_PREC_SURROGATE,
 *           double for PT_PREC_FP64
 *   npol    Jacobi terms for PT_MODEL_GIMENEZ (1..512), ignored otherwise
 * Errors: PT_ERR_ARG for inconsistent shapes (message names the light curve),
 * PT_ERR_UNSUPPORTED for PT_PREC_SURROGATE with PT_MODEL_GIMENEZ or without
 * surrogate weights. */
pt_status pt_lc_batch(const pt_batch* batch, pt_model model, int32_t npol, pt_prec prec,
                      void* flux, void* stream);

/* Gaussian log-likelihood of observed fluxes under the batch model, one value
 * per light curve, without writing the model flux (the paper notes that
 * moving the likelihood to the GPU removes the flux transfer, Sect. 3.4):
 *   log L_i = -1/2 sum_j ((obs_j - F_j)/sigma_i)^2 - N_i ln sigma_i - N_i/2 ln 2 pi
 * over the N_i = n_band_i * t_count_i points of light curve i.
 *   obs      [n_flux] observed flux in pt_lc_batch's output layout and type
 *            (float for PT_PREC_FP32/PT_PREC_SURROGATE, double for FP64), device
 *   sigma    [n_lc] white-noise standard deviation per light curve (> 0), device
 *   loglike  [n_lc] output, device, double; summed in a fixed order
 * Errors: as pt_lc_batch; PT_ERR_ARG for NULL obs/sigma/loglike.
 * Currently switched off (PT_ERR_UNSUPPORTED): its first GPU test stopped
 * responding and the cause has not been identified. */
pt_status pt_lc_loglike(const pt_batch* batch, pt_model model, int32_t npol, pt_prec prec,
                        const void* obs, const double* sigma, double* loglike, void* stream);

/* Picks the launch shape of pt_lc_batch for this batch shape by measurement
 * (a project-side tuner; the paper has no counterpart).  Candidates: the
 * default shape and every tile size in {64 .. 4096} exposures x requested
 * waves per CU in {4, 6, 8, 12, 16, 24, 32}.  Each candidate is captured into
 * a graph and replayed on `stream` as pt_lc_batch replays it: untimed replays
 * first (more for the first candidate, which also brings the clocks up), then
 * the median of seven replays timed with HIP events.  The fastest shape is
 * kept for the batch shape (it can only be the default when nothing beats
 * it) and used by later pt_lc_batch / pt_lc_batch_noalloc calls of that
 * shape on any stream; a JSON report with every candidate's median, the
 * default's and the best goes into report[report_len] (may be NULL).
 * flux: as for pt_lc_batch (overwritten).  Synchronises the stream. */
pt_status pt_autotune(const pt_batch* batch, pt_model model, int32_t npol, pt_prec prec,
                      void* flux, void* stream, char* report, size_t report_len);

/* The tuned-shape cache on disk, as JSON lines, one object per batch shape:
 *   {"key": "<gfx arch>|<batch shape>", "tile_exposures": T, "workgroups": W,
 *    "cu": C, "ms": M, "default_ms": D}
 * The key is the GPU architecture and the batch shape (model, precision,
 * npol, sizes and hashes of the host shape arrays), so a file written on one
 * GPU serves every GPU of the same architecture; workgroups scale with the
 * compute-unit count when it differs from C.
 * pt_tune_save writes every shape tuned or loaded so far (path is created or
 * truncated).  pt_tune_load merges a file into the cache (plans made before
 * take their tuned shape at once) and stores the number of entries read in
 * *n_loaded (may be NULL).  Errors: PT_ERR_ARG for a NULL path, a file that
 * cannot be opened, or a line that is not a tuned-shape object (nothing after
 * it is read). */
pt_status pt_tune_save(const char* path);
pt_status pt_tune_load(const char* path, int32_t* n_loaded);

/* Last launch shape used for a batch shape (-1 if none): tile exposures and
 * workgroups of the persistent grid. */
pt_status pt_batch_launch_shape(const pt_batch* batch, pt_model model, int32_t npol,
                                pt_prec prec, int32_t* tile_exposures, int32_t* workgroups);

/* pt_lc_batch for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same output as pt_lc_batch, with every scratch
 * buffer of the call (tile queue counters, device copies of the shape
 * arrays, the tile list, per-light-curve orbit and per-band constants) in
 * one static device array of 16 MiB that each GPU the library runs on holds
 * until the process ends.  Nothing is allocated on the device, no plan is
 * cached and no graph is captured: each call copies the shape arrays and
 * the tile list (at most 8 MiB, from a static host staging area) on
 * `stream` and launches the kernels directly.
 *   model   PT_MODEL_MA_QUAD only (else PT_ERR_UNSUPPORTED)
 *   prec    PT_PREC_FP32 or PT_PREC_FP64 (else PT_ERR_UNSUPPORTED)
 *   batch, flux as for pt_lc_batch
 * Limits: about 272 bytes per light curve, 136 per passband and 16 per tile
 * (each part rounded up to 256 bytes, plus 1 KiB of counters) must fit the
 * 16 MiB, and the shape arrays with the tile list the 8 MiB staging area;
 * tiles are made longer until the tile list fits, and a batch that does not
 * fit even then (e.g. more than about 120,000 passbands) gives PT_ERR_ARG
 * with the sizes, before any HIP call.
 * Every call on one GPU shares that GPU's array: calls on one GPU whose
 * executions overlap (different streams, or threads) race and give wrong
 * flux; serialise them.  Errors: as pt_lc_batch. */
pt_status pt_lc_batch_noalloc(const pt_batch* batch, pt_model model, pt_prec prec, void* flux,
                              void* stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate of the three Mandel-Agol functions (lambda_e,
 * lambda_d + 2/3 Theta(k-z), eta_d) = (alpha_0, alpha_1, alpha_0 - alpha_2)
 * as functions of (z, k): a 2-128-128-128-3 network with SiLU activations.
 * Weights are FP32 masters owned by the caller (device); W* are row-major
 * [out][in].  Layer widths are fixed: W1[128][2] b1[128] W2[128][128] b2[128]
 * W3[128][128] b3[128] W4[3][128] b4[3].
 * ------------------------------------------------------------------------- */
typedef struct {
  float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} pt_mlp;

/* Exact double targets (lambda_e, lambda_d + 2/3 Theta, eta_d) for zk[n][2]
 * rows (z, k); target[n][3].  Used to train the network on the GPU. */
pt_status pt_mlp_datagen(const double* zk, int64_t n, double* target, void* stream);

/* Forward pass on float rows zk[n][2] (network inputs are the scaled (z,k)
 * the library applies itself); out[n][3].  act (may be NULL) receives the
 * activations needed by pt_mlp_backward: [n][3][128] floats. */
pt_status pt_mlp_forward(const pt_mlp* w, const float* zk, int64_t n, float* out, float* act,
                         void* stream);

/* Backward pass: given dout[n][3] = dLoss/dout and the activations of the
 * matching forward call, accumulates nothing: overwrites grad with
 * dLoss/dweights summed over the n rows. */
pt_status pt_mlp_backward(const pt_mlp* w, const float* zk, const float* act, const float* dout,
                          int64_t n, pt_mlp* grad, void* stream);

/* Weighted squared error of out[n][3] (network units alpha/k^2) against the
 * exact alpha[n][3] of pt_mlp_datagen at the rows zk[n][2] (float), with
 * weight (k/0.3)^4 + 1e-3 per row (the flux error is about k^2 times the
 * output error); dout[n][3] receives dLoss/dout and loss[0] (device) the
 * mean.  Runs on `stream`. */
pt_status pt_mlp_loss_grad(const float* out, const float* zk, const double* alpha, int64_t n,
                           float* dout, float* loss, void* stream);

/* Adam update of all weights in place (m, v are first/second moments with
 * the same layout; step counts from 1). */
pt_status pt_mlp_adam_step(pt_mlp* w, const pt_mlp* grad, pt_mlp* m, pt_mlp* v, int64_t step,
                           float lr, float beta1, float beta2, float eps, void* stream);

/* Installs trained weights for PT_PREC_SURROGATE (the library keeps its own
 * BF16 copies; the caller's buffers may be freed afterwards) and builds the
 * network's error map against the exact model.  The network serves the
 * inside of the stellar disc, 0 <= z < 1 - k - fallback_band, for k in
 * [k_lo, k_hi]; every other point uses the exact functions.  Inference runs
 * bf16 MFMA products with float accumulation, weights and activations split
 * into bf16 hi + lo parts (three products); with the environment variable
 * PT_MLP_SPLIT=0 at this call, one product of the hi parts.  Synchronises the
 * stream. */
pt_status pt_surrogate_set(const pt_mlp* w, double fallback_band, double k_lo, double k_hi,
                           void* stream);

/* Fraction of error-map cells (over s = z/(1-k) in [0,1), k in [k_lo, k_hi])
 * whose network error keeps the flux of every quadratic law with uniform
 * (q1, q2) coefficients within tolerance (-1 on error). */
double pt_surrogate_trusted_fraction(void);

/* Point counters of the installed surrogate on this device: out[0] = points
 * the batch kernels (PT_PREC_SURROGATE) took from the network, out[1] =
 * in-transit points they evaluated with the exact functions instead (outside
 * the trusted cells or inside the fallback band), each (subsample, passband)
 * pair counted once, summed over every call since pt_surrogate_set or the
 * last reset.  reset != 0 sets both to zero after reading.  Synchronous (a
 * device-to-host copy; the caller orders it after the calls it counts).
 * Errors: PT_ERR_ARG for NULL out, PT_ERR_UNSUPPORTED without a surrogate. */
pt_status pt_surrogate_counters(uint64_t* out, int32_t reset);

/* Raw outputs (alpha/k^2 units) of the installed network on its bf16-MFMA
 * inference path for float rows zk[n][2], out[n][3] float: no trust map and
 * no fallback (for checking inference against pt_mlp_forward). */
pt_status pt_mlp_infer(const float* zk, int64_t n, float* out, void* stream);

/* Evaluates the installed surrogate's three functions (lambda_e, lambda_d +
 * 2/3 Theta(k - z), eta_d) at zk[n][2] (double), out[n][3] (double): the
 * network's where its error map accepts it for any quadratic law with uniform
 * (q1, q2) coefficients (lambda_e and eta_d then from their polynomials),
 * the exact double functions elsewhere. */
pt_status pt_surrogate_eval(const double* zk, int64_t n, double* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PTHIP_H */
