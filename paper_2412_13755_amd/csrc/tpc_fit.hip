// Kalman helix fit (gfx950): one thread per seed, state and covariance in
// registers, exact helix steps with analytic Jacobians, single precision.
// The hit list of a seed is read through its global cluster ids (row r of the
// seed is first_row + k, so x comes from the LDS copy of the row table and
// the map correction from [sector][row]).
#include "tpc_fit_math.hpp"
#include "tpc_internal.hpp"

namespace {

struct FitArgs {
    const int32_t *offsets, *hits, *sector, *first_row, *n_seeds;
    int32_t cap_seeds;
    const float *y, *z, *row_x, *map;
    int32_t n_rows, n_sectors, n_clusters;
    float kbz, vy, vz, max_sin, var_s, var_t, var_w;
    tpc_tracks out;
};

__global__ void __launch_bounds__(TPC_BLOCK)
fit_tracks(FitArgs A) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < A.n_rows; r += TPC_BLOCK) xs[r] = A.row_x[r];
    __syncthreads();
    int T = *A.n_seeds;
    if (T > A.cap_seeds) T = A.cap_seeds;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        const int o0 = A.offsets[i];
        const int n = A.offsets[i + 1] - o0;
        const int row0 = A.first_row[i];
        const int sec = A.sector[i];
        // a seed from tpc_ca_seed always passes these checks; others are
        // rejected instead of being read out of bounds
        const bool sane = n >= 3 && row0 >= 0 && row0 + n <= A.n_rows && sec >= 0 &&
                          sec < A.n_sectors && o0 >= 0;
        const float *mp = A.map ? A.map + (size_t)(sane ? sec : 0) * A.n_rows * 2 : nullptr;
        const int32_t *hh = A.hits + o0;
        const uint32_t NC = (uint32_t)A.n_clusters;
        auto hit_y = [&](int k, int32_t id) {
            float v = A.y[(uint32_t)id < NC ? id : 0];
            return mp ? v - mp[(row0 + k) * 2] : v;
        };
        auto hit_z = [&](int k, int32_t id) {
            float v = A.z[(uint32_t)id < NC ? id : 0];
            return mp ? v - mp[(row0 + k) * 2 + 1] : v;
        };
        float p[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        Sym5 C = {};
        float chi2 = 0.0f;
        int status = TPC_FIT_OK;
        const int ka = n - 1, kb = (n - 1) / 2;
        float xcur = sane ? xs[row0 + ka] : 0.0f;
        if (!sane) {
            status = TPC_FIT_INIT_FAIL;
        } else {
            const int32_t ia = hh[ka], ib = hh[kb], ic = hh[0];
            const float ya = hit_y(ka, ia), za = hit_z(ka, ia);
            const float yb = hit_y(kb, ib);
            const float yc = hit_y(0, ic), zc = hit_z(0, ic);
            if (!helix_start(xcur, ya, za, xs[row0 + kb], yb, xs[row0], yc, zc, A.kbz, A.max_sin, p))
                status = TPC_FIT_INIT_FAIL;
        }
        C.c00 = A.vy;
        C.c11 = A.vz;
        C.c22 = A.var_s;
        C.c33 = A.var_t;
        C.c44 = A.var_w;
        if (status == TPC_FIT_OK) {
            int32_t id_next = n >= 2 ? hh[n - 2] : 0;
            for (int k = n - 2; k >= 0; --k) {
                const int32_t id = id_next;
                if (k > 0) id_next = hh[k - 1];          // prefetch the next id
                const float my = hit_y(k, id), mz = hit_z(k, id);
                const float xk = xs[row0 + k];
                StepJac J;
                if (!helix_step(p, xk - xcur, A.kbz, A.max_sin, J)) {
                    status = TPC_FIT_SIN_FAIL;
                    break;
                }
                xcur = xk;
                cov_step(C, J);
                const float dchi = kalman_update(p, C, my, mz, A.vy, A.vz);
                if (!(dchi >= 0.0f)) {
                    status = TPC_FIT_NUM_FAIL;
                    break;
                }
                chi2 += dchi;
                if (!isfinite(chi2 + p[0] + p[1] + p[2] + p[3] + p[4])) {
                    status = TPC_FIT_NUM_FAIL;
                    break;
                }
            }
        }
        A.out.x[i] = xcur;
        float *po = A.out.par + (size_t)i * 5;
        po[0] = p[0]; po[1] = p[1]; po[2] = p[2]; po[3] = p[3]; po[4] = p[4];
        float *co = A.out.cov + (size_t)i * 15;
        co[0] = C.c00; co[1] = C.c10; co[2] = C.c11; co[3] = C.c20; co[4] = C.c21;
        co[5] = C.c22; co[6] = C.c30; co[7] = C.c31; co[8] = C.c32; co[9] = C.c33;
        co[10] = C.c40; co[11] = C.c41; co[12] = C.c42; co[13] = C.c43; co[14] = C.c44;
        A.out.chi2[i] = chi2;
        A.out.ndf[i] = 2 * n - 5;
        A.out.status[i] = status;
    }
}

}  // namespace

hipError_t launch_fit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                      const float *map, const tpc_tracks *tr, void *ws, hipStream_t st) {
    (void)ws;
    const tpc_config &c = ctx->cfg;
    FitArgs A;
    A.offsets = sd->offsets;
    A.hits = sd->hits;
    A.sector = sd->sector;
    A.first_row = sd->first_row;
    A.n_seeds = sd->n_seeds;
    A.cap_seeds = sd->cap_seeds;
    A.y = fr->y;
    A.z = fr->z;
    A.row_x = ctx->d_row_x;
    A.map = map;
    A.n_rows = c.n_rows;
    A.n_sectors = c.n_sectors;
    A.n_clusters = fr->n_clusters;
    A.kbz = -TPC_C_LIGHT * c.bz;
    A.vy = c.sigma_y * c.sigma_y;
    A.vz = c.sigma_z * c.sigma_z;
    A.max_sin = c.max_sin;
    A.var_s = c.var_sin0;
    A.var_t = c.var_tgl0;
    A.var_w = c.var_qpt0;
    A.out = *tr;
    int blocks = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fit_tracks, dim3(blocks), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}

size_t fit_ws_layout(void *ws, int64_t T) {
    (void)ws;
    (void)T;
    return 0;
}
