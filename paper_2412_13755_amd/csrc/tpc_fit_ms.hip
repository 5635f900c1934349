// Kalman fit with material (gfx950): the seed fit with multiple scattering
// in the gas as process noise and rejection of outlying hits.
//
//  fit_ms_tracks  thread per seed, double precision (plane distances and
//                 -c Bz too): three-point start at the outermost hit; for
//                 each inward step, the scattering of the segment about to
//                 be crossed enters the covariance (Highland, from the state
//                 at the plane the step leaves), then the helix step and
//                 transport; the hit's predicted-residual chi2 decides
//                 whether it is used (update) or rejected (flagged).  The
//                 next hit's coordinates are loaded a step ahead.
#include "tpc_fit_common.hpp"
#include "tpc_fit_ms.hpp"

namespace {

struct MsArgs {
    FitArgs F;
    double kbz;            // -c Bz in double precision
    double x0, mass2, cut;
    bool scatter;          // x0 finite
    uint8_t *rejected;     // [cap_hits] or null
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

__device__ inline void fit_ms_one(const MsArgs &A, int i, const float *xs) {
    const FitArgs &F = A.F;
    const SeedView sv = seed_view(F, i);
    double p[5] = {0, 0, 0, 0, 0};
    SymT<double> C = {};
    double chi2 = 0.0;
    int status = TPC_FIT_OK, used = 1;
    double xcur = sv.sane ? (double)xs[sv.row0 + sv.n - 1] : 0.0;
    if (sv.sane && A.rejected)
        for (int k = 0; k < sv.n; ++k) A.rejected[sv.o0 + k] = 0;
    if (!sv.sane) {
        status = TPC_FIT_INIT_FAIL;
    } else {
        const int ka = sv.n - 1, kb = (sv.n - 1) / 2;
        double ya, za, yb, zb, yc, zc;
        hit_meas(F, sv, ka, F.hyz ? 0 : sv.hh[ka], ya, za);
        hit_meas(F, sv, kb, F.hyz ? 0 : sv.hh[kb], yb, zb);
        hit_meas(F, sv, 0, F.hyz ? 0 : sv.hh[0], yc, zc);
        (void)zb;
        if (!helix_start<double, double>((double)xs[sv.row0 + ka], ya, za, (double)xs[sv.row0 + kb], yb,
                                         (double)xs[sv.row0], yc, zc, A.kbz, F.max_sin, p))
            status = TPC_FIT_INIT_FAIL;
    }
    C.c00 = F.vy;
    C.c11 = F.vz;
    C.c22 = F.var_s;
    C.c33 = F.var_t;
    C.c44 = F.var_w;
    if (status == TPC_FIT_OK) {
        float2 raw = hit_raw(F, sv, sv.n - 2, F.hyz ? 0 : sv.hh[sv.n - 2]);
        for (int k = sv.n - 2; k >= 0; --k) {
            double my, mz;
            hit_fix(F, sv, k, raw, my, mz);
            if (k > 0) raw = hit_raw(F, sv, k - 1, F.hyz ? 0 : sv.hh[k - 1]);
            const double xk = (double)xs[sv.row0 + k];
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
            const double S00 = C.c00 + F.vy, S01 = C.c10, S11 = C.c11 + F.vz;
            const double det = S00 * S11 - S01 * S01;
            const double chi = (r0 * (S11 * r0 - S01 * r1) + r1 * (S00 * r1 - S01 * r0)) / det;
            // (a singular S is not a rejection: the update reports it)
            if (det > 0.0 && chi > A.cut) {
                if (A.rejected) A.rejected[sv.o0 + k] = 1;
                continue;
            }
            const double dchi = kalman_update<double>(p, C, my, mz, F.vy, F.vz);
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

__global__ void __launch_bounds__(TPC_BLOCK) fit_ms_tracks(MsArgs A) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < A.F.n_rows; r += TPC_BLOCK) xs[r] = A.F.row_x[r];
    __syncthreads();
    int T = *A.F.n_seeds;
    if (T > A.F.cap_seeds) T = A.F.cap_seeds;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) fit_ms_one(A, i, xs);
}

}  // namespace

hipError_t launch_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected,
                               void *ws, hipStream_t st) {
    MsArgs A;
    A.F = make_fit_args(ctx, fr, sd, nullptr);
    A.F.out = *tr;
    if (sd->hit_yz) {
        A.F.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        float2 *hyz;
        fit_ws_layout(ws, sd->cap_seeds, sd->cap_hits, nullptr, &hyz);
        A.F.hyz = hyz;
        launch_gather(fr, sd, hyz, st);
    }
    A.kbz = -0.00299792458 * (double)ctx->cfg.bz;
    A.x0 = (double)mat->x0;
    A.scatter = mat->x0 < INFINITY;
    A.mass2 = (double)mat->mass * (double)mat->mass;
    A.cut = (double)mat->chi2_cut;
    A.rejected = rejected;
    int blocks = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fit_ms_tracks, dim3(blocks), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}
