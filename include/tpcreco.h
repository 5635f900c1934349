/*
 * tpcreco -- TPC track reconstruction on one MI355X (gfx950): neighbour
 * finding between adjacent pad rows, cellular-automaton seeding and a Kalman
 * helix fit, plus the adjoint of the summed fit chi2 with respect to a
 * per-(sector, pad row) cluster correction map.
 *
 * The paper this library follows (arXiv 2412.13755) names TPC track
 * reconstruction as the computation that fully loads the GPUs of the online
 * farm (Sec. 4.2, Sec. 5), processed one continuous-readout time frame at a
 * time with the whole frame resident in GPU memory and memory reused across
 * processing steps (Sec. 4).  It does not describe the algorithm; the
 * operations below are this library's reading, stated in each comment.
 *
 * Conventions for every call
 *   - Units: cm, GeV/c, tesla.  Coordinates are sector-local: x is the pad-row
 *     plane position, y runs along the pad row, z is the drift coordinate.
 *   - Clusters are grouped per (frame, sector, pad row): segment
 *     i = (frame * n_sectors + sector) * n_rows + row owns global cluster ids
 *     [row_offsets[i], row_offsets[i+1]).  Order within a row is arbitrary.
 *   - Every pointer inside tpc_frames, tpc_seeds and tpc_tracks and every
 *     array argument is a DEVICE pointer owned by the caller, unless the
 *     comment says "host".  The library never frees or retains them.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream) and allocate nothing: scratch memory is the caller's workspace
 *     of at least tpc_workspace_bytes() bytes, device memory, any alignment of
 *     256 bytes or more.  Nothing is synchronised unless stated.
 *   - Errors found on the host (bad arguments, short workspace) are returned
 *     before anything is enqueued.  Errors found on the device (capacity
 *     overflow) are written to the caller's device status word.
 *     tpc_last_error() gives a thread-local message for the last failure.
 */
#ifndef TPCRECO_H
#define TPCRECO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tpc_status;
#define TPC_OK               0
#define TPC_ERR_ARG         -1   /* invalid argument (null pointer, bad size, bad config) */
#define TPC_ERR_CAPACITY    -2   /* device-detected: seed or hit capacity exceeded */
#define TPC_ERR_HIP         -3   /* a HIP runtime call failed */
#define TPC_ERR_UNSUPPORTED -4   /* current device is not gfx950 */
#define TPC_ERR_WORKSPACE   -5   /* workspace missing or smaller than tpc_workspace_bytes() */

/* Per-track fit status (tpc_tracks.status). */
#define TPC_FIT_OK           0
#define TPC_FIT_INIT_FAIL    1   /* three-point start degenerate or |sin phi| >= max_sin */
#define TPC_FIT_SIN_FAIL     2   /* propagation reached |sin phi| >= max_sin */
#define TPC_FIT_NUM_FAIL     3   /* singular residual covariance or non-finite state */
#define TPC_FOLLOW_DUPLICATE 4   /* tpc_track_follow: fewer than half of its clusters are its own */
#define TPC_REFIT_NOT_HEAD   5   /* tpc_track_refit: not the head of a chain (nothing written) */
#define TPC_REFIT_LONG_CHAIN 6   /* tpc_track_refit: a chain of more than 18 segments */

/* Reconstruction constants.  Copied at tpc_create(); the context is immutable. */
typedef struct tpc_config {
    int32_t n_sectors;        /* sectors per frame, >= 1 */
    int32_t n_rows;           /* pad rows per sector, 3..256 */
    const float *row_x;       /* HOST [n_rows]: plane x of each row, strictly increasing */
    float bz;                 /* solenoid field (T), |bz| >= 1e-6 */
    float sigma_y, sigma_z;   /* cluster resolution (cm), > 0 */
    float win_y, win_z;       /* neighbour position windows (cm), > 0 */
    float cut_y, cut_z;       /* neighbour second-difference cuts (cm), > 0 */
    int32_t min_hits;         /* shortest seed kept, >= 3 */
    float max_sin;            /* |sin phi| limit of the fit, in (0, 1) */
    float var_sin0, var_tgl0, var_qpt0;   /* start covariance of sin phi, tan lambda, q/pT */
    int32_t ckpt_rows;        /* fit-state checkpoint spacing for the adjoint, 1..64 */
} tpc_config;

/* Clusters of n_frames stacked time frames. */
typedef struct tpc_frames {
    int32_t n_frames;              /* >= 1 */
    int32_t n_clusters;            /* N = row_offsets[n_frames*n_sectors*n_rows], < 2^31 */
    const int32_t *row_offsets;    /* [n_frames*n_sectors*n_rows + 1], non-decreasing, [0] = 0 */
    const float *y, *z;            /* [N] single precision */
} tpc_frames;

/* Seeds in CSR form, ordered by the global id of their first (lowest-row) hit. */
typedef struct tpc_seeds {
    int32_t cap_seeds, cap_hits;   /* capacities of the arrays below */
    int32_t *n_seeds, *n_hits;     /* device scalars: required sizes (also on overflow) */
    int32_t *offsets;              /* [cap_seeds + 1] hits of seed i: [offsets[i], offsets[i+1]) */
    int32_t *hits;                 /* [cap_hits] global cluster ids, ascending pad row */
    int32_t *frame, *sector, *first_row;   /* [cap_seeds] */
    float *hit_yz;                 /* optional [cap_hits][2], 8-byte aligned, or NULL: (y, z)
                                      of every seed hit, written by tpc_ca_seed */
} tpc_seeds;

/* Fitted tracks, one per seed (index = seed index). */
typedef struct tpc_tracks {
    float *x;                  /* [cap_seeds] plane x of the innermost hit */
    float *par;                /* [cap_seeds][5] y, z, sin phi, tan lambda, q/pT at x */
    float *cov;                /* [cap_seeds][15] covariance, packed lower triangle row by row */
    float *chi2;               /* [cap_seeds] */
    int32_t *ndf;              /* [cap_seeds] 2 n - 5 */
    int32_t *status;           /* [cap_seeds] TPC_FIT_* */
} tpc_tracks;

typedef struct tpc_context tpc_context;

/* Validates `cfg`, checks that the current HIP device is gfx950 and uploads
 * the row table (the only allocation the library makes).  The pad-row
 * planes must be equally spaced (the neighbour predicate's second
 * difference assumes it): a pitch row_x[r] - row_x[r-1] further than
 * TPC_PITCH_TOL times the mean pitch from it is refused with TPC_ERR_ARG.
 * On success *out owns a context for the current device; free it with
 * tpc_destroy(). */
#define TPC_PITCH_TOL 1e-3
tpc_status tpc_create(const tpc_config *cfg, tpc_context **out);
void tpc_destroy(tpc_context *ctx);

/* Stage bits for tpc_workspace_bytes(). */
#define TPC_STAGE_NEIGHBOURS  1
#define TPC_STAGE_SEED        2
#define TPC_STAGE_FIT         4
#define TPC_STAGE_ADJOINT     8
#define TPC_STAGE_PERSISTENT 16
#define TPC_STAGE_FOLLOW     32
#define TPC_STAGE_CTF        64
#define TPC_STAGE_SKIP      128
#define TPC_STAGE_SMOOTH    256
#define TPC_STAGE_ALL       511

/* Workspace bytes needed by the stages in `stage_mask` for frames of this
 * shape (only n_frames and n_clusters are read; host call, no device work).
 * One workspace of the returned size serves every listed stage. */
tpc_status tpc_workspace_bytes(const tpc_context *ctx, const tpc_frames *frames,
                               int32_t stage_mask, size_t *bytes);

/* Neighbour finding.  For each cluster h of row r (1 <= r <= n_rows-2) of each
 * (frame, sector), the pair (d of row r-1, u of row r+1) with
 *   |y_u - y_h| <= win_y, |z_u - z_h| <= win_z, |y_h - y_d| <= win_y,
 *   |z_h - z_d| <= win_z, |dy| <= cut_y, |dz| <= cut_z,
 *   dy = (y_u - y_h) - (y_h - y_d), dz likewise,
 * that minimises q = dy*dy + dz*dz; ties go to the smaller u id, then the
 * smaller d id.  Every operation is one IEEE single-precision rounding (no
 * fused multiply-add), so the result is exactly defined; non-finite
 * coordinates never link.  Writes up[h], dn[h] (global ids, -1 for none) for
 * every cluster, -1 in rows 0 and n_rows-1.
 * up, dn: [N] device int32, written.  ws: TPC_STAGE_NEIGHBOURS workspace. */
tpc_status tpc_neighbours(const tpc_context *ctx, const tpc_frames *frames,
                          int32_t *up, int32_t *dn, void *ws, size_t ws_bytes, void *stream);

/* Neighbour finding across one missing pad row (pad-row inefficiency, dead
 * rows) -- a variant of the search above that the paper does not describe.
 * Partners may lie one or two rows away: d in row r-a, u in row r+b, a and b
 * in {1, 2}, both rows inside the sector.  With A = y_u - y_h, B = y_h - y_d
 * (z likewise) a triplet passes if |A| <= b win, |B| <= a win (y and z with
 * their windows) and |D| <= cut for D = g (A/b - B/a), g = 2/(a+b): the
 * divided second difference at unit row pitch, 0 on a straight line, the
 * same on a parabola for every (a, b), and the dy above at a = b = 1.  The
 * triplet spanning the fewest rows wins (a+b = 2, then 3, then 4), then the
 * smallest q = Dy^2 + Dz^2, then the smaller u id, then the smaller d id;
 * so a cluster keeps its adjacent-row result whenever it has one.  One IEEE
 * single-precision rounding per operation (A/b, B/a and b win exact, g =
 * 2/3 rounded once).  Output as tpc_neighbours.  ws: TPC_STAGE_SKIP
 * workspace (the neighbour workspace plus a list of queried clusters).  The
 * links feed tpc_ca_seed unchanged, and its seeds then skip rows: fit them
 * with tpc_kalman_fit_rows (tpc_kalman_fit assumes consecutive rows). */
tpc_status tpc_neighbours_skip(const tpc_context *ctx, const tpc_frames *frames,
                               int32_t *up, int32_t *dn, void *ws, size_t ws_bytes, void *stream);

/* Cellular-automaton seeding from the neighbour links.
 *   links   h -> up[h] is kept if dn[up[h]] == h (and symmetrically);
 *   chains  maximal runs of kept links, bottom b to top t, m >= 2 clusters;
 *   claims  a chain with m >= min_hits-2 claims dn[b] and up[t] when these are
 *           in no chain; each claimed cluster goes to the smallest (-m, b);
 *   seeds   [dn[b] if won] + chain + [up[t] if won], kept with >= min_hits
 *           clusters, ordered by the global id of their first cluster.
 * up, dn: [N] from tpc_neighbours.  seeds: caller arrays and capacities.
 * dev_status: device int32, set to TPC_OK or TPC_ERR_CAPACITY (then
 * the counters n_seeds and n_hits hold the required sizes and the arrays
 * hold a prefix).
 * When seeds->hit_yz is not NULL, the (y, z) of every placed seed hit is
 * copied there from the frames, in seed-hit order, by the workgroups that
 * place the hits (coalesced reads of the frames); the fit and the adjoint
 * then read hit coordinates from it instead of gathering them by id.
 * ws: TPC_STAGE_SEED workspace. */
tpc_status tpc_ca_seed(const tpc_context *ctx, const tpc_frames *frames,
                       const int32_t *up, const int32_t *dn, tpc_seeds *seeds,
                       int32_t *dev_status, void *ws, size_t ws_bytes, void *stream);

/* Seeding without any allocation, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation): tpc_ca_seed with its workspace taken from a
 * library-owned device array of TPC_NOALLOC_SCRATCH_BYTES per device
 * (reserved when the library's code is loaded on that device and held until
 * the process ends; its address is looked up once per device by
 * tpc_create).  Arguments, results and device status as tpc_ca_seed; no
 * workspace argument.  Frames whose seeding workspace
 * (tpc_workspace_bytes with TPC_STAGE_SEED) exceeds the array are refused
 * with TPC_ERR_WORKSPACE before anything is enqueued (128 MiB: about 2.7 M
 * clusters over 36 x 152 segments).  The current device must be the
 * context's.  Every call on a device uses that device's one array, whose
 * contents persist between calls (the kernels initialise every word they
 * read): calls that overlap in time on one device race and must be ordered
 * by the caller, e.g. issued on one stream. */
#define TPC_NOALLOC_SCRATCH_BYTES (128u << 20)
tpc_status tpc_ca_seed_noalloc(const tpc_context *ctx, const tpc_frames *frames,
                               const int32_t *up, const int32_t *dn, tpc_seeds *seeds,
                               int32_t *dev_status, void *stream);

/* Kalman helix fit of every seed (count read on the device from *n_seeds,
 * clamped to cap_seeds).  State (y, z, sin phi, tan lambda, q/pT) on the
 * pad-row planes, curvature -0.00299792458 * bz * q/pT per cm; start: exact
 * circle through the outermost, middle and innermost hits at the outermost
 * hit with covariance diag(sigma_y^2, sigma_z^2, var_sin0, var_tgl0,
 * var_qpt0); then for each hit inwards an exact helix step with its analytic
 * Jacobian (no process noise) and a Kalman update with the hit.  chi2 is the
 * sum of the predicted-residual chi2, ndf = 2n - 5.  The state, Jacobian,
 * covariance and update are carried in double precision; outputs are single
 * precision.  Hit coordinates come from seeds->hit_yz when it is not NULL
 * (it must then hold the coordinates of `frames`, as tpc_ca_seed writes
 * them), else from frames->y/z by hit id.
 * map: optional [n_sectors][n_rows][2] (dy, dz) subtracted from every
 * cluster of that (sector, row) before fitting (NULL = none).
 * ckpt: optional device buffer of >= tpc_ckpt_bytes() bytes (8-byte
 * aligned); when given, the filter state every ckpt_rows updates is stored
 * there for tpc_fit_adjoint().  ws: TPC_STAGE_FIT workspace. */
tpc_status tpc_kalman_fit(const tpc_context *ctx, const tpc_frames *frames,
                          const tpc_seeds *seeds, const float *map, tpc_tracks *tracks,
                          void *ckpt, size_t ckpt_bytes, void *ws, size_t ws_bytes, void *stream);

/* Fit with material: tpc_kalman_fit (no map, no checkpoints) plus multiple
 * scattering in the gas as process noise and the rejection of outlying
 * hits -- a variant of the fit the paper's reconstruction implies but does
 * not describe.  Before each inward step from plane a to plane b (state p at
 * a), the scattering of that segment enters the covariance: path
 * ds = |x_b - x_a| sqrt(1 + t^2) / sqrt(1 - s^2), momentum P = sqrt(1 + t^2)/|w|,
 * beta = P / sqrt(P^2 + mass^2), theta0 = 0.0136 / (beta P) sqrt(ds/x0)
 * (1 + 0.038 ln(ds/x0)) (Highland), th2 = theta0^2:
 *   C_ss += th2 (1 - s^2)(1 + t^2), C_tt += th2 (1 + t^2)^2,
 *   C_tw += th2 t w (1 + t^2), C_ww += th2 t^2 w^2
 * (none for x0 infinite or w = 0).  With rho > 0 the segment's energy loss
 * follows: the particle moves outwards, so the step inwards gives back the
 * mean loss ds rho <dE/dx> at fixed direction (Bethe formula, unit charge,
 * no density term: <dE/dx> = K Z/A / beta^2 (ln(2 m_e beta^2 gamma^2 W /
 * I^2)/2 - beta^2), W the largest energy transfer, K = 0.307075 MeV cm^2/mol),
 * E' = E + loss, P' = sqrt(E'^2 - mass^2), w' = w P/P'; the straggling
 * (Bohr, relativistic: var E = K Z/A rho ds m_e (1 - beta^2/2)/(1 - beta^2))
 * enters C_ww as var E (w E/P^2)^2, and C <- J C J^T with J the map's
 * Jacobian in (t, w) at fixed loss.  A segment whose loss would change P by
 * more than 1 % is taken without it; a particle that would stop ends the
 * fit with TPC_FIT_SIN_FAIL.  After the helix step, a hit whose
 * predicted-residual chi2 exceeds chi2_cut is not used: the filter goes on
 * from the prediction and rejected[seed hit] = 1 (else 0).  chi2 sums the
 * used hits; ndf = 2 (used hits + 1) - 5, the outermost (start) hit
 * counted.  Double precision throughout.  mat: host pointer; x0 > 0 (cm,
 * infinity = no scattering), mass >= 0 (GeV), chi2_cut > 0 (infinity = keep
 * all), rho >= 0 (g/cm^3, 0 = no energy loss; with rho > 0 also mass > 0,
 * z_over_a > 0 (mol/g) and mean_exc > 0 (GeV), all finite, else
 * TPC_ERR_ARG).  rejected: optional device uint8 [cap_hits].  ws:
 * TPC_STAGE_FIT workspace. */
typedef struct tpc_material {
    float x0;
    float mass;
    float chi2_cut;
    float rho;
    float z_over_a;
    float mean_exc;
} tpc_material;
tpc_status tpc_kalman_fit_material(const tpc_context *ctx, const tpc_frames *frames,
                                   const tpc_seeds *seeds, const tpc_material *mat,
                                   tpc_tracks *tracks, uint8_t *rejected, void *ws, size_t ws_bytes,
                                   void *stream);

/* Fit of seeds whose hits may skip pad rows, with per-cluster errors.  The
 * pad row of each hit is the row of the seed's (frame, sector) whose id
 * range holds it (seeds->first_row is not read); a seed with a hit outside
 * that (frame, sector), or whose rows do not rise strictly with the hit
 * index, gets status TPC_FIT_INIT_FAIL and zero outputs.  Hit h is
 * measured with variances cluster_err[2h]^2, cluster_err[2h+1]^2 (its
 * sigma_y, sigma_z in cm, also the start covariance at the outermost hit);
 * cluster_err NULL: the configured sigma_y, sigma_z for every hit.  mat as
 * for tpc_kalman_fit_material, NULL for no scattering and no rejection (the
 * plain fit over the hits' own rows).  Otherwise as tpc_kalman_fit_material.
 * cluster_err: optional device float [n_clusters][2], 8-byte aligned.
 * rejected: optional device uint8 [cap_hits].  ws: TPC_STAGE_FIT workspace. */
tpc_status tpc_kalman_fit_rows(const tpc_context *ctx, const tpc_frames *frames,
                               const tpc_seeds *seeds, const float *cluster_err,
                               const tpc_material *mat, tpc_tracks *tracks, uint8_t *rejected,
                               void *ws, size_t ws_bytes, void *stream);

/* The fit over rows (tpc_kalman_fit_rows, same arguments and outputs), then
 * a smoother giving the state at every seed hit's plane from all hits --
 * part of the two-pass fitting that the paper's reconstruction implies but
 * does not describe.  Reference: the fit's final state carried by exact
 * helix steps to every plane.  About it the problem is linear in the
 * deviation d = state - reference: a Kalman filter of d runs inwards from
 * the outermost hit (d = 0, variances (100 sigma)^2 on y and z and var_sin0,
 * var_tgl0, var_qpt0), with the step Jacobians and the scattering noise of
 * mat taken on the reference and the hits the fit used (not those it
 * rejected); then the Rauch-Tung-Striebel pass outwards,
 *   G = C_k F^T P^-1,  P = F (C_k + Q) F^T,
 *   d_s(k) = d_k + G (d_s(k-1) - F d_k),  C_s(k) = C_k + G (C_s(k-1) - P) G^T.
 * hit_par[h][5] and hit_cov[h][15] (packed like tracks->cov) receive the
 * smoothed state reference + d_s and its covariance at seed hit h's plane,
 * in seed-hit order; zeros for seeds whose fit failed.  A failing smoother
 * step sets the track's status to TPC_FIT_SIN_FAIL or TPC_FIT_NUM_FAIL.
 * Double precision throughout, single-precision outputs.
 * rejected, hit_par, hit_cov: device, [cap_hits], [cap_hits][5],
 * [cap_hits][15], required.  ws: TPC_STAGE_SMOOTH workspace (the fit's,
 * plus 5 doubles per seed and 20 doubles + 2 bytes per seed hit). */
tpc_status tpc_kalman_smooth(const tpc_context *ctx, const tpc_frames *frames,
                             const tpc_seeds *seeds, const float *cluster_err,
                             const tpc_material *mat, tpc_tracks *tracks, uint8_t *rejected,
                             float *hit_par, float *hit_cov, void *ws, size_t ws_bytes, void *stream);

/* Checkpoint-buffer bytes for seeds of these capacities (host call). */
tpc_status tpc_ckpt_bytes(const tpc_context *ctx, const tpc_seeds *seeds, size_t *bytes);

/* loss (device float scalar) = sum of chi2 over tracks with status
 * TPC_FIT_OK, accumulated in double precision in a fixed order
 * (bit-reproducible).  ws: TPC_STAGE_FIT workspace. */
tpc_status tpc_chi2_sum(const tpc_context *ctx, const tpc_seeds *seeds, const tpc_tracks *tracks,
                        float *loss, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of L(M) = sum of chi2 over tracks with status TPC_FIT_OK with
 * respect to the correction map M [n_sectors][n_rows][2] used in the fit:
 * grad_map = dloss * dL/dM, through the start, the helix steps (including
 * the dependence of each Jacobian on the state), the gains and the chi2.
 * Seeds stay fixed.  Requires the checkpoints of a tpc_kalman_fit() call
 * with the same frames, seeds and map; tracks.status comes from that call.
 * Reverse mode: each ckpt_rows-step segment is recomputed from its
 * checkpoint, then run backwards.  Per-row sums are formed in a fixed order,
 * so the result is bit-reproducible.  dloss: device float scalar (NULL = 1).
 * grad_map: [n_sectors][n_rows][2] device floats, overwritten.
 * ws: TPC_STAGE_ADJOINT workspace (sized for the default capacities
 * cap_hits = N and cap_seeds = N / min_hits + 1; larger capacities need more,
 * reported as TPC_ERR_WORKSPACE). */
tpc_status tpc_fit_adjoint(const tpc_context *ctx, const tpc_frames *frames,
                           const tpc_seeds *seeds, const float *map, const tpc_tracks *tracks,
                           const void *ckpt, size_t ckpt_bytes, const float *dloss,
                           float *grad_map, void *ws, size_t ws_bytes, void *stream);

/* Whole path (tpc_neighbours, tpc_ca_seed, tpc_kalman_fit without map or
 * checkpoints) for all n_frames frames of `frames`; results are identical in
 * every mode.
 *   TPC_MODE_STAGED      the three stage calls one after another (several
 *                        kernel launches per stage)
 *   TPC_MODE_PERSISTENT  neighbours and seeding in one persistent kernel on
 *                        a grid of workgroups that are resident at once,
 *                        moving through the phases with grid-wide barriers,
 *                        then the fit as one launch over the seeds longest
 *                        first (plus small initialisation and status
 *                        kernels).  If the grid cannot synchronise (a
 *                        barrier wait exceeds its bounded polling), every
 *                        workgroup leaves and *dev_status is set to
 *                        TPC_ERR_HIP.
 *   TPC_MODE_PERSISTENT_GRAPH  the persistent sequence captured once into a
 *                        HIP graph held by the context (keyed by every
 *                        argument: frames, buffers, workspace, tune) and
 *                        replayed on `stream` by later calls with the same
 *                        arguments; the first call with new arguments
 *                        captures on a stream of the context's own and
 *                        instantiates the graph (host-side allocation),
 *                        replays allocate nothing.  The buffers must stay
 *                        valid while the context keeps the graph (until
 *                        tpc_destroy).
 * tune: NULL or { grid: workgroups (0 = resident capacity, larger values are
 * clamped to it), sort_fit: 1 = longest seeds first, 0 = seed order,
 * fit_block: workgroup size of the fit (0 = 256; 64, 128 or 256),
 * fit_spt: about this many seeds per fit thread (0 = 1; at most 64) }.
 * grid and sort_fit apply to the persistent modes, the fit shape to all.
 * The staged and persistent modes are graph-capturable (no allocation, no
 * host synchronisation).
 * ws: TPC_STAGE_NEIGHBOURS|SEED|FIT workspace (staged) or
 * TPC_STAGE_PERSISTENT workspace (persistent). */
#define TPC_MODE_STAGED      0
#define TPC_MODE_PERSISTENT  1
#define TPC_MODE_PERSISTENT_GRAPH 2
typedef struct tpc_tune {
    int32_t grid;
    int32_t sort_fit;
    int32_t fit_block;
    int32_t fit_spt;
} tpc_tune;
tpc_status tpc_reconstruct(const tpc_context *ctx, const tpc_frames *frames, int32_t mode,
                           const tpc_tune *tune, int32_t *up, int32_t *dn, tpc_seeds *seeds,
                           tpc_tracks *tracks, int32_t *dev_status, void *ws, size_t ws_bytes,
                           void *stream);

/* Track following: the step after the fit that the paper's reconstruction
 * implies but does not describe (Sec. 4.2 names track reconstruction as the
 * load of the farm's GPUs); this is a textbook prolongation with cluster
 * pickup.  For every seed i (double precision throughout, no map):
 *   0  the fit of tpc_kalman_fit (state at the innermost hit);
 *   A  inwards, pad row by pad row below the innermost hit: helix step to the
 *      row; stop if it fails or |y| > x tan 10 deg (the track leaves the
 *      sector); take the cluster of that (frame, sector, row) with the
 *      smallest chi2 of its predicted residual, r^T (C_yz + diag(sigma_y^2,
 *      sigma_z^2))^-1 r, ties to the smaller id; if chi2 <= gate_chi2 update
 *      the state with it, else count a miss, and stop after more than
 *      max_miss consecutive misses;
 *   B  outwards: restart at the innermost hit (its measured y, z, the other
 *      parameters from A, the fit's start covariance), update with every hit
 *      above it up to the outermost, then prolong outwards as in A;
 *   C  refit all hits exactly as tpc_kalman_fit does a seed (three-point start
 *      at the outermost, middle ((n-1)/2 in ascending row order) and
 *      innermost hits; steps across empty rows go plane to plane).
 * A cluster may be taken by several tracks.  Then duplicates: every cluster
 * belongs to the track of smallest key (n_rows - n_hits, index) among the
 * tracks with status TPC_FIT_OK holding it; a track owning fewer than half
 * of its clusters gets status TPC_FOLLOW_DUPLICATE (broken pieces of one
 * particle's chain grow into the same track and only one is kept).
 * params: host pointer; gate_chi2 finite, >= 0; max_miss in 0..n_rows.
 * rows: [cap_seeds][n_rows] device int32, written for i < *n_seeds: the
 * cluster of track i in each pad row, -1 where it has none.
 * tracks: as tpc_kalman_fit, for the refit (ndf = 2 n_hits - 5), status
 * TPC_FIT_* of the seed fit or the refit, or TPC_FOLLOW_DUPLICATE.
 * Seeds are read as tpc_ca_seed writes them (hit_yz is not used).
 * ws: TPC_STAGE_FOLLOW workspace. */
typedef struct tpc_follow_params {
    float gate_chi2;
    int32_t max_miss;
} tpc_follow_params;
tpc_status tpc_track_follow(const tpc_context *ctx, const tpc_frames *frames,
                            const tpc_seeds *seeds, const tpc_follow_params *params,
                            int32_t *rows, tpc_tracks *tracks, void *ws, size_t ws_bytes,
                            void *stream);

/* Merging of fitted segments across sector edges (the continuation of track
 * following across sectors, which the paper's reconstruction implies but
 * does not describe).  A particle crossing from one sector into the next on
 * the same side leaves a fitted segment in each.  For segments A, B of one
 * frame in neighbouring sectors of one side (36-sector geometry only),
 * both with status TPC_FIT_OK, A's innermost point (x, y) at the smaller
 * radius: A's state is rotated into B's frame (turned by the sectors' angle
 * difference da: a point (x, y) -> (x cos da + y sin da, -x sin da + y cos
 * da), phi -> phi - da, cos phi > 0 required) and carried along the helix
 * to B's plane x; chi2 = d^T (J C_A J^T + C_B)^-1 d with d the state
 * difference and J the transfer's Jacobian (in FP64).  A's best outer
 * partner is the B of smallest chi2 <= chi2_cut (smaller index on ties), B's
 * best inner partner likewise; when each is the other's best, next[A] = B,
 * prev[B] = A and chi2[A] = the pair's chi2; otherwise -1 and 0.  Seeds must
 * be ordered by (frame, sector), as tpc_ca_seed writes them.  tracks: as a
 * fit writes them, one per seed.  next, prev, chi2: device [cap_seeds]
 * (int32, int32, float); the first min(*n_seeds, cap_seeds) are written.
 * merged_par [cap_seeds][5], merged_cov [cap_seeds][15] (device float, both
 * or neither may be NULL): for a linked A the pair refitted as one at B's
 * plane, in B's frame -- A's transferred state (covariance P = J C_A J^T)
 * and B's, independent fits of disjoint hits, combined: x = p_A' +
 * P S^-1 (p_B - p_A'), C = P S^-1 C_B, S = P + C_B (the joint fit of both
 * segments' hits for the linearised problem); zeros where unlinked.
 * leg [cap_seeds] (int32), leg_chi2 [cap_seeds] (float), both or neither
 * NULL: the legs of loopers.  A returning leg is fitted as a track running
 * outwards along the same circle in the other sense (same centre, curvature
 * and tan(lambda) of opposite signs).  Per segment m = (X_c, Y_c, kappa,
 * tan(lambda)), the circle centre in global coordinates (kappa = -c Bz q/pT);
 * two fitted segments of one frame and side (any sectors), both with circle
 * radius below 250 cm, compare by chi2 = d^T (J_A C_A J_A^T + D J_B C_B J_B^T
 * D)^-1 d, d = m_A - D m_B, D = diag(1, 1, -1, -1); mutual best partners
 * with chi2 <= chi2_cut (smaller index on ties) get leg[A] = B, leg[B] = A;
 * else -1 and 0.  chi2_cut > 0 and finite, else TPC_ERR_ARG. */
tpc_status tpc_track_merge(const tpc_context *ctx, const tpc_seeds *seeds, const tpc_tracks *tracks,
                           float chi2_cut, int32_t *next, int32_t *prev, float *chi2, float *merged_par,
                           float *merged_cov, int32_t *leg, float *leg_chi2, void *stream);

/* Tracks assembled from linked segments and refitted over all their hits
 * (the step after merging; the paper implies it but does not describe it).
 * Links: a next link i -> j counts when j = next[i] is another segment with
 * prev[j] = i and both segment fits (segments->status) are TPC_FIT_OK; a leg
 * link i -- j when leg[j] = i likewise (leg NULL: none).  next, prev and leg
 * are read as tpc_track_merge writes them.
 * track_id [cap_seeds] (device int32): the connected components of the
 * segments of status TPC_FIT_OK under both kinds of link, each named by its
 * smallest segment index; -1 for a segment whose own fit failed.
 * refit: as a fit writes tracks, one entry per segment.  A chain head (status
 * TPC_FIT_OK, no counted prev link) gets the refit of its chain -- the head
 * and the segments its next links reach, at most 18 (else
 * TPC_REFIT_LONG_CHAIN) -- over all their hits k = 0..n-1 (the head's in
 * ascending row, then the next segment's, ...), each measured in its own
 * sector's frame and corrected by `map` as tpc_kalman_fit does: the exact
 * circle through hits n-1, (n-1)/2 and 0, all seen from the frame of hit n-1
 * (a point (x, y) of a sector at angle a_s seen from the frame at angle a_t:
 * (x cos d - y sin d, x sin d + y cos d), d = a_s - a_t, sector angles as in
 * tpc_track_merge), starts the filter at hit n-1 with the start covariance;
 * it runs inwards, a helix step within a segment and, across a segment
 * boundary, the rotation into the inner segment's frame and the step on to
 * its plane (the transfer of tpc_track_merge, covariance J C J^T), each
 * followed by the update.  Written at the head: the state at its innermost
 * hit in its frame, chi2, ndf = 2n - 5, status TPC_FIT_*.  Every other
 * segment gets status TPC_REFIT_NOT_HEAD and zeros.  A chain of one segment
 * is refitted exactly as its seed fit.
 * loop_par [cap_seeds][4], loop_cov [cap_seeds][10] (packed lower
 * triangle), loop_chi2 [cap_seeds] (device float; all three or none, and
 * none when leg is NULL): for each counted leg link i -- j with i < j whose
 * chains' refits have status TPC_FIT_OK, the joint circle of the two legs
 * at index i: the circles m = (X_c, Y_c, kappa, tan lambda) of the two
 * refitted chains at their heads (as tpc_track_merge's legs), fused in the
 * sense of i's chain: S = S_i + D S_j D, d = m_i - D m_j, m = m_i - S_i S^-1
 * d, C = S_i S^-1 D S_j D, chi2 = d^T S^-1 d; elsewhere zeros and chi2 -1.
 * Seeds are read as tpc_ca_seed writes them from adjacent-row links: hit j of
 * a seed lies in row first_row + j, as tpc_kalman_fit reads them (hit_yz is
 * not used); a segment whose rows leave 0..n_rows-1 or whose hit ids leave
 * the frames makes its chain's status TPC_FIT_INIT_FAIL.  The first
 * min(*n_seeds, cap_seeds) entries of each output are written.  No
 * workspace. */
tpc_status tpc_track_refit(const tpc_context *ctx, const tpc_frames *frames, const tpc_seeds *seeds,
                           const tpc_tracks *segments, const int32_t *next, const int32_t *prev,
                           const int32_t *leg, const float *map, int32_t *track_id, tpc_tracks *refit,
                           float *loop_par, float *loop_cov, float *loop_chi2, void *stream);

/* Entropy coding of a time frame's integer arrays (Sec. 4.1: every flat
 * integer array is coded on its own with range asymmetric numeral systems,
 * the symbol distribution counted for each frame, several coders
 * interleaved on one stream).  This library's coder:
 *   frequencies  counts c_s over the array's range [lo, hi] (R = hi - lo + 1
 *                <= 2^20 entries, D symbols present, D <= 2^L), scaled to
 *                M = 2^L: f_s = floor(c_s (M - D) / n) + 1 where c_s > 0,
 *                else 0; the shortfall M - sum f goes to the most frequent
 *                symbol (the smallest on ties);
 *   coder        32-bit state in [2^16, 2^32), 16-bit words: to code s, if
 *                x >= f_s 2^(32-L) emit x mod 2^16 and shift x right by 16,
 *                then x <- floor(x / f_s) 2^L + (x mod f_s) + cum_s;
 *   interleaving blocks of B symbols; symbol 64 j + k of a block belongs to
 *                coder k (64 coders starting at 2^16); a block is coded
 *                backwards (j, then k, descending) onto one word stack;
 *   stream       little-endian: u32 magic 0x534E4152, u32 version 2, u64 n,
 *                i32 lo, u32 R, u32 L, u32 B, u32 blocks, u32 T; the
 *                frequency table in T bytes, zero-padded to a multiple of 4;
 *                u32 word_start[blocks + 1] (in words); u32 state[blocks][64];
 *                u16 words, each block's stack last pushed first;
 *   table        compressed, as the paper does with the decoding metadata:
 *                for each present symbol in ascending order, the run of
 *                absent symbols before it and f - 1, each an unsigned LEB128
 *                varint (7 bits a byte, low group first, high bit on all but
 *                the last byte; at most 3 bytes).
 * A decoder runs each block forwards: slot = x mod 2^L, s with
 * cum_s <= slot < cum_s + f_s, x <- f_s (x >> L) + slot - cum_s, and while
 * x < 2^16, x <- x 2^16 + next word. */
#define TPC_RANS_LANES 64
typedef struct tpc_rans_params {
    int32_t scale_bits;       /* L, 1..16 */
    int32_t block_symbols;    /* B, a multiple of 64, 64..2^24 */
} tpc_rans_params;

/* Workspace bytes of tpc_rans_encode for n symbols (host call). */
tpc_status tpc_rans_workspace_bytes(int64_t n, const tpc_rans_params *params, size_t *bytes);

/* Largest stream for n symbols whose range is at most `range` (host call):
 * 40 + (6 min(range, 2^16) rounded up to 4) + 4 (blocks + 1) + 256 blocks
 * + 2 n bytes (no range when n = 0). */
tpc_status tpc_rans_max_bytes(int64_t n, int64_t range, const tpc_rans_params *params, size_t *bytes);

/* Codes symbols[0..n) (device int32, 0 <= n < 2^31) into out (device, 4-byte
 * aligned, out_cap bytes).  *out_size (device u64) receives the stream's
 * exact size.  *dev_status (device int32) receives TPC_OK, TPC_ERR_ARG (range
 * wider than 2^20 or more than 2^L distinct symbols; nothing written) or
 * TPC_ERR_CAPACITY (the stream is larger than out_cap; nothing written,
 * *out_size says how large).  The output is identical for identical input
 * (integer arithmetic throughout).  ws: tpc_rans_workspace_bytes() bytes. */
tpc_status tpc_rans_encode(const int32_t *symbols, int64_t n, const tpc_rans_params *params,
                           void *out, size_t out_cap, uint64_t *out_size, int32_t *dev_status,
                           void *ws, size_t ws_bytes, void *stream);

/* Track-model residual transform: a frame's clusters as flat integer
 * arrays for the entropy coder (Sec. 4.1 reduces every detector's time
 * frame to integer arrays and codes each on its own; the arrays below are
 * this library's reading for the TPC).  Q(v) = rint(v * (1/q)) in single
 * precision (1/q rounded to float), 0 when not finite or beyond +-2^30.
 * Each cluster belongs to the lowest-index track with status TPC_FIT_OK
 * (after tpc_track_follow) holding it, else it is free.  Per such track, in
 * index order: trk_seg = frame * n_sectors + sector, trk_n = its own
 * clusters, trk_row0 = the first one's pad row, Q(y0), Q(z0) split into
 * v >> 8 (trk_y0h, trk_z0h) and v & 255 (trk_y0l, trk_z0l), trk_dy1 =
 * Q(y1) - Q(y0), trk_dz1 likewise (0 for fewer clusters); per own cluster
 * k >= 1 in row order, hit_drow = r_k - r_(k-1) - 1; per k >= 2, hit_ry =
 * Q(y_k) - 2 Q(y_(k-1)) + Q(y_(k-2)), hit_rz likewise.  Per segment (frame,
 * sector, row): seg_nfree = its free clusters, whose Q(y), Q(z) follow in
 * id order split the same way (free_yh, free_yl, free_zh, free_zl).
 * rows, tracks: the output of tpc_track_follow for these seeds.  q_y, q_z:
 * host floats > 0.  out: device arrays of cap_seeds (trk_*), n_clusters
 * (hit_*, free_*) and n_frames*n_sectors*n_rows (seg_nfree) entries;
 * out->counts (device int64[TPC_CTF_ARRAYS]) receives the number of entries
 * written to each array, in the order of the struct.  ws: TPC_STAGE_CTF
 * workspace (sized for the default seed capacity N / min_hits + 1; larger
 * capacities need more, reported as TPC_ERR_WORKSPACE). */
#define TPC_CTF_ARRAYS 17
typedef struct tpc_ctf_arrays {
    int32_t *trk_seg, *trk_n, *trk_row0, *trk_y0h, *trk_y0l, *trk_z0h, *trk_z0l, *trk_dy1, *trk_dz1;
    int32_t *hit_drow, *hit_ry, *hit_rz;
    int32_t *seg_nfree;
    int32_t *free_yh, *free_yl, *free_zh, *free_zl;
    int64_t *counts;
} tpc_ctf_arrays;
tpc_status tpc_ctf_build(const tpc_context *ctx, const tpc_frames *frames, const tpc_seeds *seeds,
                         const int32_t *rows, const tpc_tracks *tracks, float q_y, float q_z,
                         const tpc_ctf_arrays *out, void *ws, size_t ws_bytes, void *stream);

/* Decodes a stream of tpc_rans_encode (device, 4-byte aligned, `size`
 * bytes) into symbols (device int32, capacity `cap` < 2^31).  *n_out (device
 * int64) receives the stream's symbol count; *dev_status (device int32)
 * TPC_OK, TPC_ERR_CAPACITY (more symbols than cap; nothing written) or
 * TPC_ERR_ARG (malformed: bad header or version, a table varint longer than 3
 * bytes or cut off, an odd number of varints, a symbol past the range,
 * frequencies not summing to 2^L, a block not returning its coders to 2^16
 * or not using exactly its words;
 * the symbols written are then meaningless).  Every read is bounds-checked
 * against `size`.  ws: tpc_rans_decode_workspace_bytes() bytes. */
tpc_status tpc_rans_decode_workspace_bytes(size_t *bytes);
tpc_status tpc_rans_decode(const void *in, size_t size, int32_t *symbols, int64_t cap, int64_t *n_out,
                           int32_t *dev_status, void *ws, size_t ws_bytes, void *stream);

/* Several arrays (1..TPC_RANS_BATCH_MAX) coded by one set of launches, each
 * exactly as tpc_rans_encode would (same parameters for all).  An array's
 * symbol count is n, or, when n_device is not NULL, the device int64 it
 * points to clamped to 0..n (n is then the capacity; the counts of
 * tpc_ctf_build can be passed without a host synchronisation).  Each job
 * has its own output, size and status as in tpc_rans_encode.
 * ws: tpc_rans_batch_workspace_bytes() bytes (which reads n only). */
#define TPC_RANS_BATCH_MAX 24
typedef struct tpc_rans_job {
    const int32_t *symbols;
    int64_t n;
    const int64_t *n_device;
    void *out;
    size_t out_cap;
    uint64_t *out_size;
    int32_t *dev_status;
} tpc_rans_job;
tpc_status tpc_rans_batch_workspace_bytes(int32_t count, const tpc_rans_job *jobs,
                                          const tpc_rans_params *params, size_t *bytes);
tpc_status tpc_rans_encode_batch(int32_t count, const tpc_rans_job *jobs, const tpc_rans_params *params,
                                 void *ws, size_t ws_bytes, void *stream);

/* Workgroups the persistent kernel can keep resident on the context's device. */
int32_t tpc_persistent_grid(const tpc_context *ctx);

/* Status code name. */
const char *tpc_status_string(tpc_status s);
/* Thread-local description of the last failure in this thread ("" if none). */
const char *tpc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
