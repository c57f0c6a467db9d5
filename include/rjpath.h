/*
 * rjpath.h -- C ABI of librjpath.so: batched reversible-jump MCMC sampling of
 * photon paths from a point source to a spherical light sensor through a
 * scattering and absorbing medium, on AMD Instinct MI355X (gfx950).
 *
 * Method: G. H. Collin, "Using path integrals for the propagation of light in
 * a scattering dominated medium", arXiv:1811.04156.  A path is a polyline
 * f_0 .. f_{n-1} (Sec. "Numerical path integration"); its density is the
 * factorised product of the appendix ("Path probability distribution"):
 *   p = p_i(f_0,f_1) prod_{k=1}^{n-2} p_v(f_{k-1},f_k,f_{k+1}) p_f(f_{n-2},f_{n-1}).
 * Chains move by single-vertex perturbations and by birth/death jumps through
 * the bi-spherical dimension-matching map (App. "Jump proposal", "Dimension
 * matching transformation"), accepted with Green's reversible-jump ratio
 * (eq. acceptFact).  The detected intensity is the integral of p over all
 * paths (Sec. "Comparison of relative light yield" motivates it; the
 * estimator used here anchors one sector by quadrature).
 *
 * Conventions shared by every call:
 *  - Every array argument marked "device" is a device pointer owned by the
 *    caller; "host" arrays are read during the call only.  The library owns
 *    only the opaque rjpath_medium handle and the workspaces inside it.
 *  - Calls return RJPATH_OK (0) or a negative error code; they never throw.
 *    rjpath_last_error() returns a thread-local message for the last failure.
 *    Argument errors are detected on the host before any work is enqueued.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    rjpath_run_chains and rjpath_grad are asynchronous; rjpath_intensity
 *    synchronises the stream because its finalisation runs on the host.
 *  - Lengths are metres.  Media are given as scattering length lambda_s and
 *    absorption length lambda_a (b = 1/lambda_s, a = 1/lambda_a; an infinite
 *    length means a zero coefficient) and the mean scattering cosine g.
 */
#ifndef RJPATH_H
#define RJPATH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RJPATH_OK = 0,
    RJPATH_EINVAL = -1,  /* invalid argument (message says which) */
    RJPATH_ENOMEM = -2,  /* device allocation failed (init / workspace growth only) */
    RJPATH_EHIP = -3,    /* a HIP runtime call failed (message has the HIP error) */
    RJPATH_ENODATA = -4, /* a target has no anchor-sector visits yet */
    RJPATH_ENOTSUP = -5  /* combination not supported by this build */
};

enum { RJPATH_F32 = 0, RJPATH_F64 = 1 };              /* element type of path vertices */
/* interior-vertex move: Gaussian step; joint Langevin move of all interior
 * vertices; single-vertex Langevin move; tree-coordinate move of the whole
 * path on the first step of every cycle (Gaussian steps otherwise) */
enum { RJPATH_PLAIN = 0, RJPATH_MALA = 1, RJPATH_LMALA = 2, RJPATH_TREE = 3 };
enum { RJPATH_EMIT_ISO = 0, RJPATH_EMIT_VMF = 1, RJPATH_EMIT_CONE = 2 };
enum { RJPATH_DET_UNIFORM = 0, RJPATH_DET_PAPER = 1 };

/* Per-chain statistics, RJPATH_NSTAT doubles per chain, added to by every
 * post-burn-in step (step index >= burn_in):
 *  0 samples              1 sum 1/w(n)             2 sum [n == n0] / w(n0)
 *  3 sum path length L    4 sum L^2                 5 sum n
 *  6 proposed perturb     7 proposed birth          8 proposed death
 *  9 accepted perturb    10 accepted birth         11 accepted death
 * 12 steps at n == cap   13 proposed Langevin or tree move   14 accepted Langevin or tree move
 * 15 jumps rejected without a density evaluation (birth at cap, death at n = 2) */
enum { RJPATH_NSTAT = 16 };

/* Per-step trace record (tests): 5 doubles per chain and step:
 * move (0 interior, 1 end point, 2 birth, 3 death, 4 joint Langevin, 5 none,
 * 6 single-vertex Langevin, 7 tree-coordinate move of the whole path),
 * accepted (0/1), index (vertex or segment, -1 if none), log A, log u. */
enum { RJPATH_TRACE_WORDS = 5 };

typedef struct rjpath_medium rjpath_medium;

/* Layered media (App. "Intermediate vertex": a(x), b(x), sigma(cos theta)).
 * Medium m has layer_cnt[m] layers along the unit axis axis[3m..3m+2];
 * its edges are edges[layer_off[m] + m .. layer_off[m] + m + layer_cnt[m]]
 * (strictly increasing), layer l covers [edge_l, edge_{l+1}) and the first and
 * last layers extend to -inf / +inf.  Per-layer arrays are indexed by
 * layer_off[m] + l.  f_sl is the simplified-Liu fraction of the scattering
 * function (eq. angular_scattering); 0 gives pure Henyey-Greenstein.
 * All arrays are host memory. */
typedef struct {
    int32_t n_media;
    const double* axis;
    const int32_t* layer_off;
    const int32_t* layer_cnt;
    const double* edges;
    const double* lam_s;
    const double* lam_a;
    const double* g;
    const double* f_sl;
} rjpath_medium_desc;

/* Source/sensor pairs ("targets"); every array is device memory, T entries.
 *  medium[T]       medium index
 *  src[3T]         absolute point-source position (App. "Initial vertex")
 *  sensor[3T]      absolute centre of the spherical sensor (App. "Final vertex")
 *  radius[T]       sensor radius
 *  emit_kind[T]    RJPATH_EMIT_*: isotropic; von Mises-Fisher (eq. emission_dist,
 *                  emit_param = kappa); uniform cone (emit_param = half-angle, rad)
 *  emit_dir[3T]    preferred emission direction (unit)
 *  emit_param[T]
 *  det_kind[T]     RJPATH_DET_*: rho = 1, or eq. (detection_prob) with det_dir
 *  det_dir[3T]     preferred sensor direction rho_hat (unit)
 *  n0[T]           anchor sector (2 or 3) of the intensity estimator
 *  logw            NULL, or T*(cap+1) sector tilts log w(n) (the chain samples
 *                  p(f) w(n); the intensity estimator undoes the tilt)       */
typedef struct {
    int32_t n_targets;
    const int32_t* medium;
    const double* src;
    const double* sensor;
    const double* radius;
    const int32_t* emit_kind;
    const double* emit_dir;
    const double* emit_param;
    const int32_t* det_kind;
    const double* det_dir;
    const int32_t* n0;
    const double* logw;
} rjpath_targets;

/* Chain state, all device memory.  Vertex v of chain c is element
 * verts[v * n_chains + c], four values (x, y, z, w) of the precision's type:
 * x, y, z relative to the chain's source (f_0 = 0), w is library-owned scratch
 * (the scattering depth of the segment leaving the vertex).  Slots v >= n[c]
 * are unused.  logp[c] receives log p of the final path; status[c] is 0 for a
 * healthy chain and 1 if its starting path had zero or non-finite density
 * (such a chain is not moved and adds nothing to the statistics).
 * work: proposal buffer with the layout of verts (required for RJPATH_MALA
 * and RJPATH_TREE, else may be NULL). */
typedef struct {
    int32_t n_chains;
    int32_t cap;       /* maximum vertex count, 2 <= cap <= 4096 */
    int32_t precision; /* RJPATH_F32 or RJPATH_F64 */
    const int32_t* target;
    int32_t* n;
    void* verts;
    double* logp;
    int32_t* status;
    double* stats; /* n_chains * RJPATH_NSTAT */
    void* work;
} rjpath_chains;

/* Run parameters.  The random draws of chain c at global step s are two
 * Philox4x32-10 blocks with counter (c, s mod 2^32, s >> 32, 0 / 1) and key
 * (seed mod 2^32, seed >> 32); MALA vertex k uses counter word 3 = 2 + k.
 * Step s is a perturbation step if (s mod cycle_len) < n_perturb, else a jump
 * step that is a birth when draw 2 < birth_thresh and a death otherwise
 * (birth_thresh = birth fraction * 2^32).  Steps run from step0 to
 * step0 + steps - 1; statistics accumulate for steps >= burn_in.
 * sigma: standard deviation (m) of the Gaussian interior-vertex step;
 * kappa_end: concentration of the von Mises-Fisher end-point step on the
 * sensor; sampler: RJPATH_PLAIN; RJPATH_MALA (interior steps become joint
 * Langevin moves of all interior vertices with step size mala_h, m^2); or
 * RJPATH_LMALA (an interior step moves vertex j by a Langevin step
 * y_j = f_j + (h/2) d log p / d f_j + sqrt(h) xi with the dimensionless
 * mala_h scaling h = mala_h * min(|f_j - f_{j-1}|, |f_{j+1} - f_j|)^2; the
 * Discussion's suggestion of gradient-informed moves); or RJPATH_TREE (step s
 * with s mod cycle_len == 0 moves the whole path in the tree coordinates of
 * App. "Path space coordinate system": the end point by the von
 * Mises-Fisher step and every interior vertex's bi-spherical coordinates
 * (zeta = artanh cos s, t, phi) about its foci by Gaussian steps of variance
 * mala_h / n, Sec. "Path proposal distribution"; vertex k draws one Philox
 * block with counter word 3 = 2 + k; the other perturbation steps are
 * Gaussian steps sigma).
 * block_chains (multiple of 64) and v_lds (vertex slots per chain kept in
 * LDS; each chain's LDS tile also holds two padding slots, so
 * (v_lds + 2) * block_chains vertices must fit the LDS left after the media
 * tables, else RJPATH_EINVAL) select the launch; 0 takes the values tuned for
 * this handle (see rjpath_autotune) or a default.  chunk: steps per kernel launch (0 = all).
 * trace: NULL or n_chains * steps * RJPATH_TRACE_WORDS doubles.
 * hist: NULL or n_targets * (cap + 1) uint32 counts (added to) of the sector n
 * after every step of the call, burn-in included (for tuning the sector tilt).
 * step_counter: NULL, or a device uint64 holding the global step index; the
 * kernels then read the first step from it (step0 is ignored) and the call
 * enqueues an increment by `steps` after them.  A captured graph of the call
 * (hipStreamBeginCapture / torch.cuda.graph) then advances the chains on
 * every replay instead of repeating the same random numbers.  Such a call
 * records kernel nodes only (no memset), and trace must be NULL. */
typedef struct {
    uint64_t seed;
    uint64_t step0;
    int64_t burn_in;
    int32_t steps;
    int32_t cycle_len;
    int32_t n_perturb;
    uint32_t birth_thresh;
    double sigma;
    double kappa_end;
    int32_t sampler;
    double mala_h;
    int32_t block_chains;
    int32_t v_lds;
    int32_t chunk;
    double* trace;
    uint32_t* hist;
    uint64_t* step_counter;
} rjpath_run_params;

/* One candidate of rjpath_tune_proposal: the proposal parameters of
 * rjpath_run_params it replaces. */
typedef struct {
    double sigma;
    double kappa_end;
    double mala_h;
    int32_t cycle_len;
    int32_t n_perturb;
} rjpath_proposal;

/* Thread-local description of the last error. */
const char* rjpath_last_error(void);

/* Library version string. */
const char* rjpath_version(void);

/* Builds the device tables of one or more layered media (per layer: a, b,
 * log b, Henyey-Greenstein and simplified-Liu constants, the concentration
 * kappa_eq with coth(k) - 1/k = g of the birth centering rule (App. "Dimension
 * matching transformation"), prefix integrals of a and b along the axis).
 * Allocates device memory (the only call besides rjpath_autotune that does).
 * Errors: RJPATH_EINVAL for n_media < 1, an empty medium, lambda <= 0 or NaN,
 * |g| >= 1, f_sl outside [0,1], unsorted edges or a non-unit axis. */
int rjpath_init_medium(rjpath_medium** out, const rjpath_medium_desc* desc, void* stream);

/* Releases the handle and its device memory (NULL is a no-op). */
int rjpath_free_medium(rjpath_medium* m);

/* Advances every chain by p->steps reversible-jump steps in place and adds
 * the per-chain statistics (see RJPATH_NSTAT) into c->stats.  Deterministic
 * given (seed, step0): the same state and parameters give bit-identical
 * results for any launch configuration.  Paths are clamped to n <= cap (a
 * birth at cap is a rejected proposal).  Allocates nothing. */
int rjpath_run_chains(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c,
                      const rjpath_run_params* p, void* stream);

/* Anchor integrals I_{n0} per target (host output, T doubles): the integral
 * of p over the anchor sector, by product Gauss quadrature on the device in
 * FP64.  n0 = 2: over the directions from the source into the sensor
 * (dOmega = cos Phi dA / r^2, App. "Final vertex"); n0 = 3: one scattering
 * vertex, integrated over emission directions and, along each ray, layer by
 * layer between the layer edges it crosses.  Independent of the chains; the
 * result can be reused while media and targets are unchanged.
 * Synchronises `stream`; may grow a workspace inside the handle. */
int rjpath_anchor(rjpath_medium* m, const rjpath_targets* t, double* anchor, void* stream);

/* Detected intensity per target from the chain statistics, with the anchored
 * sector estimator  I = I_{n0} * sum_c stats[1] / sum_c stats[2].
 * anchor: host array of the T anchors from rjpath_anchor, or NULL to have
 * them computed in this call.  Standard error by delete-one-group jackknife
 * over `groups` chain groups of each target (a chain's group is a hash of
 * its index; 2 <= groups <= 64).  Host outputs (each T doubles, any may be
 * NULL): I, se, ess = (I/se)^2, rhat = potential scale reduction of the path
 * length over the groups (Sec. "Implementation").  Synchronises `stream`;
 * may grow a workspace inside the handle.
 * Errors: RJPATH_ENODATA if a target with chains has no anchor-sector
 * visits (its outputs are NaN; the others are still written). */
int rjpath_intensity(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t groups,
                     const double* anchor, double* I, double* se, double* ess, double* rhat, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rjpath_intensity with no
 * allocation, no host synchronisation and no copy.  Its reduction buffer
 * (and the anchors, when `anchor` is NULL) live in a static device array of
 * 512 Ki doubles (4 MiB) per GPU, held until the process ends; it requires
 * n_targets * groups * 6 (+ n_targets when anchor is NULL) <= 524288, else
 * RJPATH_EINVAL.  anchor: NULL (computed here) or device, n_targets doubles.
 * I, se, ess, rhat: device, n_targets doubles each (any may be NULL), written
 * by a device finalisation identical in arithmetic to rjpath_intensity's; a
 * target without anchor-sector visits gets NaN (no RJPATH_ENODATA, since
 * nothing is read back).  Asynchronous on `stream`.  Every call on one GPU
 * uses that GPU's one buffer: calls that overlap on a GPU (other streams,
 * other threads) race and must be serialised by the caller. */
int rjpath_intensity_noalloc(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t groups,
                             const double* anchor, double* I, double* se, double* ess, double* rhat, void* stream);

/* Relative light yield B = I_1 / I_0 of two sensors lit by one source
 * (Sec. "Comparison of relative light yield"), by the geometric bridge
 * estimator  B = E_0[sqrt(q_1 / q_0)] / E_1[sqrt(q_0 / q_1)]  with
 * q_0(x) = p_0(x) and q_1(x) = p_1(T x) |dT/dx| for paths x ending on sensor 0,
 * where T bends a path toward sensor 1 along a cylinder tangent to the
 * emission axis at the source (App. "Relative light yield transformation";
 * interior vertex Jacobian b1^2 Omega (r_C + xbar b1) / b0^3, end point moved
 * rigidly by the rotation of the arrival frames and scaled by R1 / R0).
 * This call adds one sample per chain from the chains' current paths (a
 * snapshot; call it between runs, e.g. every few hundred steps):
 *  pairs  device, 2 * n_pairs targets (t0, t1): same source position, same
 *         medium; t0's emission direction gives the cylinder's tangent
 *  role   device, n_targets: 2 k + side for a target of pair k (side 0 for t0,
 *         1 for t1), -1 for a target in no pair (each target in at most one pair)
 *  acc    device, n_pairs * 2 * groups * 2 doubles, ADDED to:
 *         acc[((k * 2 + side) * groups + g) * 2 + 0] += sqrt(r) / w(n),
 *         acc[... + 1] += 1 / w(n) over the chains of chain group g (the
 *         intensity estimator's hash) with status 0, where r = q_1(x) / q_0(x)
 *         for a chain on t0 (0 where T x leaves the map's domain) and
 *         r = q_0(x) / q_1(x) at x = T^-1 y for a chain on t1 (path y)
 *  logr   device, n_chains doubles, or NULL: log r of each chain (NaN for
 *         chains in no valid pair)
 * The tilt 1/w(n) makes tilted chains estimate untilted expectations (T
 * keeps the vertex count).  A pair whose targets differ in source or medium,
 * or whose geometry has no cylinder (sensor 1 on the emission axis), adds
 * nothing.  Asynchronous on `stream`; allocates nothing. */
int rjpath_yield_accumulate(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t n_pairs,
                            const int32_t* pairs, const int32_t* role, int32_t groups, double* acc, double* logr,
                            void* stream);

/* B and its standard error (delete-one-group jackknife, the group deleted on
 * both sides) per pair from the sums of rjpath_yield_accumulate.  acc: device;
 * B, se: host, n_pairs doubles each (either may be NULL).  Synchronises
 * `stream`.  RJPATH_ENODATA if a pair has no samples on a side or no overlap
 * (its outputs are NaN; the others are still written). */
int rjpath_yield(int32_t n_pairs, int32_t groups, const double* acc, double* B, double* se, void* stream);

/* Path-length histogram of the current paths per target (the arrival-time
 * distribution at a sensor is that of L / c in a bulk of constant index;
 * Sec. "Comparison of timing distributions"): for each chain with status 0,
 * hist[t * (bins + 1) + b] += 1 / w(n) where b = floor((L - l0) / bin_width)
 * lies in [0, bins), and hist[t * (bins + 1) + bins] += 1 / w(n) always, so
 * that the normalised histogram of p is hist[t][b] / hist[t][bins].
 * L = sum of segment lengths, summed in FP64.  hist: device,
 * n_targets * (bins + 1) doubles, added to.  Asynchronous; allocates nothing. */
int rjpath_length_hist(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, int32_t bins, double l0,
                       double bin_width, double* hist, void* stream);

/* Score of the current paths, recomputed from the vertices (no stored tape):
 *  logp_out[C]      (device, may be NULL): log p of each path, FP64 sum
 *  dlogp_dv         (device, may be NULL): d log p / d vertex, layout of verts,
 *                   precision of the chains; w component 0; vertex 0 gets 0
 *  score            (device, may be NULL): n_targets * (1 + 3 * L_total)
 *                   doubles ADDED to: [t][0] += sum_c 1/w(n_c) and
 *                   [t][1 + 3 l + k] += sum_c (1/w(n_c)) d log p / d theta_{l,k}
 *                   for global layer index l and theta = (lambda_s, lambda_a, g),
 *                   over the chains of target t with status 0.
 * Since I = int p, d log I / d theta = E_p[d log p / d theta] = score[t][1+..] / score[t][0]
 * averaged over samples (App. "Path probability distribution" gives log p). */
int rjpath_grad(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, double* logp_out,
                void* dlogp_dv, double* score, void* stream);

/* Length-weighted score sums of the current paths, for the gradient of the
 * mean path length (the arrival-time delay that constrains scattering, Sec.
 * "Comparison of timing distributions"): score_L (device, n_targets *
 * (1 + 3 * L_total) doubles, the layout of rjpath_grad's score) is ADDED to:
 * [t][0] += L_c / w(n_c) and [t][1 + 3 l + k] += (L_c / w(n_c)) d log p / d theta_{l,k}
 * over the chains of target t with status 0, where L_c is the path length.
 * Asynchronous on `stream`; allocates nothing. */
int rjpath_score_length(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, double* score_L,
                        void* stream);

/* Mean path length m_t = E_p[L] = score_L[t][0] / score[t][0] and its gradient
 * d m_t / d theta_j = E_p[L s_j] - E_p[L] E_p[s_j] (s = d log p / d theta, the
 * derivative of a normalised expectation) from the sums of rjpath_grad (score)
 * and rjpath_score_length (score_L) accumulated over the same paths.
 * mean_L: device, n_targets doubles (may be NULL); dmean_L: device,
 * n_targets * 3 L_total doubles (theta = lambda_s, lambda_a, g per global
 * layer); NaN for a target without samples.  Asynchronous on `stream`. */
int rjpath_dlength_dtheta(rjpath_medium* m, const rjpath_targets* t, const double* score, const double* score_L,
                          double* mean_L, double* dmean_L, void* stream);

/* Sector-tilt tuning (the tilt w(n) of the anchored estimator; the estimator
 * undoes it, so any tilt leaves the intensity unchanged, but a flat sector
 * histogram lets distant targets visit the anchor sector n0 often).
 * Runs `rounds` pilot rounds of p->steps sampler steps each, starting at
 * p->step0 (ordinary steps: the chains advance by rounds * p->steps steps;
 * the per-chain statistics are left untouched).  After each round, for every
 * target, log w(n) is raised by log(h(mode) / h(n)) for n0 <= n < mode, where
 * h is that round's sector histogram and mode its most visited sector (by
 * floor_push where h(n) = 0), and clamped to [0, max_logw].
 * t->logw: device, n_targets * (cap + 1) doubles, updated in place (required).
 * hist: device workspace of n_targets * (cap + 1) uint32; holds the last
 * round's histogram on return.  p->step_counter and p->trace must be NULL.
 * Asynchronous on `stream`; allocates nothing. */
int rjpath_tune_tilt(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                     int32_t rounds, uint32_t* hist, double max_logw, double floor_push, void* stream);

/* d log I_t / d theta from the score sums of rjpath_grad (the score identity
 * of the path integral, App. "Path probability distribution"):
 * dlogI[t][3 l + k] = score[t][1 + 3 l + k] / score[t][0] for the global layer
 * index l and theta = (lambda_s, lambda_a, g); NaN for a target without
 * samples.  score: device, n_targets * (1 + 3 L_total) doubles; dlogI: device,
 * n_targets * 3 L_total doubles.  Asynchronous on `stream`. */
int rjpath_dlogi_dtheta(rjpath_medium* m, const rjpath_targets* t, const double* score, double* dlogI, void* stream);

/* Times short launches of rjpath_run_chains over the candidate launch
 * configurations (the default launch, and chains per block in {64, 256} x
 * LDS vertex slots in {8, 12, 16, 24, 32}, capped at cap and at 160 KiB of
 * LDS; at most 11) on the
 * given chains, advancing them by exactly `steps` steps starting at p->step0
 * (ordinary sampler steps, so they may serve as burn-in: the chain trajectory
 * does not depend on the launch configuration), and stores the fastest
 * configuration in the handle for this (cap, precision, sampler).  Writes it to
 * best_block_chains / best_v_lds if non-NULL.  `steps` must be at least the
 * twice the number of candidates (each is timed in two passes, the second in
 * reverse order).  Synchronises the stream. */
int rjpath_autotune(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c,
                    const rjpath_run_params* p, int32_t steps, int32_t* best_block_chains, int32_t* best_v_lds,
                    void* stream);

/* Picks the proposal parameters (interior step sigma, end-point
 * concentration kappa_end, Langevin step mala_h, and the move mix
 * n_perturb / cycle_len) that give the intensity estimator the most effective
 * samples per second: each candidate runs `trial_steps` ordinary sampler steps
 * from p (two passes over the candidates, the second in reverse order, so the
 * chains advance by 2 * n_cand * trial_steps steps from p->step0), with its
 * statistics in a buffer of its own (c->stats is untouched); its score is
 * 1 / (median over targets of (se / I)^2 x seconds per trial), where se / I is
 * the jackknife relative error over `groups` chain groups of that trial's
 * estimator ratio.  Every candidate kernel leaves the path density invariant,
 * so the trials may serve as burn-in.  score: host, n_cand doubles or NULL;
 * best: host, the index of the highest score.  Allocates (the trial
 * statistics) and synchronises `stream`. */
int rjpath_tune_proposal(rjpath_medium* m, const rjpath_targets* t, const rjpath_chains* c, const rjpath_run_params* p,
                         int32_t n_cand, const rjpath_proposal* cand, int32_t trial_steps, int32_t groups,
                         double* score, int32_t* best, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RJPATH_H */
