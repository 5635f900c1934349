// Kalman fit with material (gfx950): the seed fit with multiple scattering
// in the gas as process noise and rejection of outlying hits; the same
// kernel also fits seeds whose hits skip pad rows, with per-cluster errors.
//
//  fit_ms_tracks  thread per seed, double precision (plane distances and
//                 -c Bz too): three-point start at the outermost hit; for
//                 each inward step, the scattering of the segment about to
//                 be crossed enters the covariance (Highland, from the state
//                 at the plane the step leaves), then the helix step and
//                 transport; the hit's predicted-residual chi2 decides
//                 whether it is used (update) or rejected (flagged).  The
//                 next hit's coordinates are loaded a step ahead.
//                 ROWS: the pad row of every hit is looked up in the
//                 cluster layout of the seed's (frame, sector) -- a binary
//                 search for the outermost hit, then a walk down from the
//                 row above for each next one (at most R + n reads of the
//                 row offsets per seed, all within the seed's R + 1) -- and
//                 a seed whose rows do not rise strictly, or with a hit
//                 outside its (frame, sector), is refused before the fit.
//                 ERRS: hit h is measured with variances err[h]^2.
#include "tpc_fit_common.hpp"
#include "tpc_fit_ms.hpp"

namespace {

struct MsArgs {
    FitArgs F;
    double kbz;            // -c Bz in double precision
    double x0, mass2, cut;
    bool scatter;          // x0 finite
    uint8_t *rejected;     // [cap_hits] or null
    // fits over any rows
    const int32_t *row_offsets;   // cluster layout of the frames
    const int32_t *frame;         // frame of each seed
    int32_t n_frames;
    const float2 *err;            // per-cluster (sigma_y, sigma_z), cm
};

// Adds the scattering of a segment of plane distance dx to C (state p at
// the plane the segment starts from).
__device__ inline void add_scattering(const MsArgs &A, const double p[5], double dx, SymT<double> &C) {
    const double s = p[2], t = p[3], w = p[4];
    if (!A.scatter || w == 0.0) return;
    const double t2 = 1.0 + t * t;
    const double ds = fabs(dx) * sqrt(t2) / sqrt(1.0 - s * s);
    const double pm = sqrt(t2) / fabs(w);
    const double beta = pm / sqrt(pm * pm + A.mass2);
    const double xr = ds / A.x0;
    const double th = 0.0136 / (beta * pm) * sqrt(xr) * (1.0 + 0.038 * log(xr));
    const double th2 = th * th;
    C.c22 += th2 * (1.0 - s * s) * t2;
    C.c33 += th2 * t2 * t2;
    C.c43 += th2 * t * w * t2;
    C.c44 += th2 * t * t * w * w;
}

// Row of cluster id at or below row r_hi of a (frame, sector) whose R + 1
// row offsets are ro: walking down from r_hi, the first row starting at or
// before id; -1 if id is not in that row (it lies above r_hi, or below the
// first row).
__device__ inline int walk_row(const int32_t *ro, int r_hi, int32_t id) {
    int r = r_hi;
    while (r >= 0 && ro[r] > id) --r;
    return (r >= 0 && id < ro[r + 1]) ? r : -1;
}

// Rows of the outermost, middle ((n-1)/2) and innermost hits of a seed, if
// every hit lies in the (frame, sector) and the rows rise strictly.
__device__ inline bool seed_rows(const int32_t *ro, int R, const SeedView &sv, int &ra, int &rb, int &rc) {
    const int n = sv.n, kb = (n - 1) / 2;
    const int32_t top = sv.hh[n - 1];
    if (top < ro[0] || top >= ro[R]) return false;
    int lo = 0, hi = R - 1;                       // ro[lo] <= top < ro[hi + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ro[mid] <= top) lo = mid;
        else hi = mid - 1;
    }
    int r = lo;
    ra = rb = r;
    for (int k = n - 2; k >= 0; --k) {
        r = walk_row(ro, r - 1, sv.hh[k]);
        if (r < 0) return false;
        if (k == kb) rb = r;
    }
    rc = r;
    return true;
}

template <bool ROWS, bool ERRS>
__device__ inline void fit_ms_one(const MsArgs &A, int i, const float *xs) {
    static_assert(ROWS || !ERRS, "per-cluster errors come with the row lookup");
    const FitArgs &F = A.F;
    SeedView sv = seed_view(F, i);
    const int32_t *ro = nullptr;
    int ra = 0, rb = 0, rc = 0;                   // rows of hits n-1, (n-1)/2, 0
    bool refused = false;
    if (ROWS) {
        // the layout gives the rows; first_row is not read
        const int32_t fi = A.frame[i];
        const bool inb = sv.n >= 3 && sv.o0 >= 0 && sv.o0 <= F.cap_hits - sv.n;
        if (inb && A.rejected)
            for (int k = 0; k < sv.n; ++k) A.rejected[sv.o0 + k] = 0;
        sv.sane = inb && sv.sec >= 0 && sv.sec < F.n_sectors && fi >= 0 && fi < A.n_frames;
        if (sv.sane) {
            ro = A.row_offsets + ((size_t)fi * F.n_sectors + sv.sec) * F.n_rows;
            sv.sane = seed_rows(ro, F.n_rows, sv, ra, rb, rc);
        }
        refused = !sv.sane;
    } else {
        if (sv.sane) {
            ra = sv.row0 + sv.n - 1;
            rb = sv.row0 + (sv.n - 1) / 2;
            rc = sv.row0;
        }
        if (sv.sane && A.rejected)
            for (int k = 0; k < sv.n; ++k) A.rejected[sv.o0 + k] = 0;
    }
    double p[5] = {0, 0, 0, 0, 0};
    SymT<double> C = {};
    double chi2 = 0.0;
    int status = TPC_FIT_OK, used = 1;
    double xcur = sv.sane ? (double)xs[ra] : 0.0;
    double vy = F.vy, vz = F.vz;
    if (ERRS && sv.sane) {
        const float2 e = A.err[sv.hh[sv.n - 1]];
        vy = (double)e.x * (double)e.x;
        vz = (double)e.y * (double)e.y;
    }
    if (!sv.sane) {
        status = TPC_FIT_INIT_FAIL;
    } else {
        const int ka = sv.n - 1, kb = (sv.n - 1) / 2;
        double ya, za, yb, zb, yc, zc;
        hit_meas(F, sv, ka, F.hyz ? 0 : sv.hh[ka], ya, za);
        hit_meas(F, sv, kb, F.hyz ? 0 : sv.hh[kb], yb, zb);
        hit_meas(F, sv, 0, F.hyz ? 0 : sv.hh[0], yc, zc);
        (void)zb;
        if (!helix_start<double, double>((double)xs[ra], ya, za, (double)xs[rb], yb, (double)xs[rc], yc, zc,
                                         A.kbz, F.max_sin, p))
            status = TPC_FIT_INIT_FAIL;
    }
    if (!refused) {
        C.c00 = vy;
        C.c11 = vz;
        C.c22 = F.var_s;
        C.c33 = F.var_t;
        C.c44 = F.var_w;
    }
    if (status == TPC_FIT_OK) {
        float2 raw = hit_raw(F, sv, sv.n - 2, F.hyz ? 0 : sv.hh[sv.n - 2]);
        int rk = ra;
        for (int k = sv.n - 2; k >= 0; --k) {
            double my, mz;
            hit_fix(F, sv, k, raw, my, mz);
            if (k > 0) raw = hit_raw(F, sv, k - 1, F.hyz ? 0 : sv.hh[k - 1]);
            if (ROWS) {
                rk = walk_row(ro, rk - 1, sv.hh[k]);     // valid: checked by seed_rows
            } else {
                rk = sv.row0 + k;
            }
            if (ERRS) {
                const float2 e = A.err[sv.hh[k]];
                vy = (double)e.x * (double)e.x;
                vz = (double)e.y * (double)e.y;
            }
            const double xk = (double)xs[rk];
            const double dx = xk - xcur;
            add_scattering(A, p, dx, C);
            StepJac J;
            if (!helix_step<double, double>(p, dx, A.kbz, F.max_sin, J)) {
                status = TPC_FIT_SIN_FAIL;
                break;
            }
            sym_transport<double, false>(C, J);
            xcur = xk;
            // predicted-residual chi2 of the hit
            const double r0 = my - p[0], r1 = mz - p[1];
            const double S00 = C.c00 + vy, S01 = C.c10, S11 = C.c11 + vz;
            const double det = S00 * S11 - S01 * S01;
            const double chi = (r0 * (S11 * r0 - S01 * r1) + r1 * (S00 * r1 - S01 * r0)) / det;
            // (a singular S is not a rejection: the update reports it)
            if (det > 0.0 && chi > A.cut) {
                if (A.rejected) A.rejected[sv.o0 + k] = 1;
                continue;
            }
            const double dchi = kalman_update<double>(p, C, my, mz, vy, vz);
            chi2 += dchi;
            const double chk = chi2 + p[0] + p[1] + p[2] + p[3] + p[4];
            if (!(dchi >= 0.0) || !(chk - chk == 0.0)) {
                status = TPC_FIT_NUM_FAIL;
                break;
            }
            ++used;
        }
    }
    F.out.x[i] = (float)xcur;
    float *po = F.out.par + (size_t)i * 5;
    for (int q = 0; q < 5; ++q) po[q] = (float)p[q];
    float *co = F.out.cov + (size_t)i * 15;
    const double cc[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                           C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    for (int q = 0; q < 15; ++q) co[q] = (float)cc[q];
    F.out.chi2[i] = (float)chi2;
    F.out.ndf[i] = 2 * used - 5;
    F.out.status[i] = status;
}

template <bool ROWS, bool ERRS>
__global__ void __launch_bounds__(TPC_BLOCK) fit_ms_tracks(MsArgs A) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < A.F.n_rows; r += TPC_BLOCK) xs[r] = A.F.row_x[r];
    __syncthreads();
    int T = *A.F.n_seeds;
    if (T > A.F.cap_seeds) T = A.F.cap_seeds;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        fit_ms_one<ROWS, ERRS>(A, i, xs);
}

MsArgs make_ms_args(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const tpc_material *mat,
                    const tpc_tracks *tr, uint8_t *rejected, void *ws, hipStream_t st) {
    MsArgs A;
    A.F = make_fit_args(ctx, fr, sd, nullptr);
    A.F.out = *tr;
    if (sd->hit_yz) {
        A.F.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        float2 *hyz;
        fit_ws_layout(ws, sd->cap_seeds, sd->cap_hits, nullptr, &hyz);
        A.F.hyz = hyz;
        (void)launch_gather(fr, sd, hyz, st);    // a launch error surfaces at the fit's launch
    }
    A.kbz = -0.00299792458 * (double)ctx->cfg.bz;
    A.x0 = mat ? (double)mat->x0 : (double)INFINITY;
    A.scatter = mat && mat->x0 < INFINITY;
    A.mass2 = mat ? (double)mat->mass * (double)mat->mass : 0.0;
    A.cut = mat ? (double)mat->chi2_cut : (double)INFINITY;
    A.rejected = rejected;
    A.row_offsets = fr->row_offsets;
    A.frame = sd->frame;
    A.n_frames = fr->n_frames;
    A.err = nullptr;
    return A;
}

int fit_blocks(const tpc_seeds *sd) {
    int blocks = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace

hipError_t launch_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected,
                               void *ws, hipStream_t st) {
    const MsArgs A = make_ms_args(ctx, fr, sd, mat, tr, rejected, ws, st);
    hipLaunchKernelGGL((fit_ms_tracks<false, false>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_fit_rows(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const float *err,
                           const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected, void *ws,
                           hipStream_t st) {
    MsArgs A = make_ms_args(ctx, fr, sd, mat, tr, rejected, ws, st);
    A.err = reinterpret_cast<const float2 *>(err);
    if (err)
        hipLaunchKernelGGL((fit_ms_tracks<true, true>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    else
        hipLaunchKernelGGL((fit_ms_tracks<true, false>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}
