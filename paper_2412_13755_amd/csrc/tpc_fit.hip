// Kalman helix fit (gfx950): one thread per seed, state and covariance in
// registers (covariance algebra in FP64, Jacobian in FP32; see
// tpc_fit_math.hpp), exact helix steps with analytic Jacobians.  Hits of a
// seed are read through their global cluster ids; row r of the seed is
// first_row + k, so x comes from an LDS copy of the row table and the map
// correction from [sector][row].  Optionally writes filter-state checkpoints
// every ckpt_rows updates for the adjoint.
#include "tpc_fit_common.hpp"

namespace {

__device__ inline void fit_all(const FitArgs &A) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < A.n_rows; r += blockDim.x) xs[r] = A.row_x[r];
    __syncthreads();
    int T = *A.n_seeds;
    if (T > A.cap_seeds) T = A.cap_seeds;
    if (A.order) {
        const int n = *A.n_order;
        T = n < T ? n : T;
    }
    // grid-stride: a launch of g workgroups of b threads fits every seed
    // with ceil(T / (g b)) seeds per thread (the launch shape is a tuning
    // knob; results do not depend on it)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < T; i += gridDim.x * blockDim.x) {
        const int s = A.order ? A.order[i] : i;
        if ((uint32_t)s < (uint32_t)A.cap_seeds) fit_one(A, s, xs);
    }
}

// Seeds in seed order (the fit stage).
__global__ void __launch_bounds__(TPC_BLOCK)
fit_tracks(FitArgs A) {
    fit_all(A);
}

// The fit in length order (the staged fit of many seeds, or after the
// persistent kernel with sort_fit): the same code under its own name, so
// profiles tell the launches apart.
__global__ void __launch_bounds__(TPC_BLOCK)
fit_tracks_ordered(FitArgs A) {
    fit_all(A);
}

// (y, z) of every seed hit in seed-hit order, so the fit reads each seed's
// measurements contiguously instead of through the id indirection.
__global__ void __launch_bounds__(TPC_BLOCK)
gather_hits(const int32_t *__restrict__ n_hits, int32_t cap_hits, const int32_t *__restrict__ hits,
            const float *__restrict__ y, const float *__restrict__ z, int32_t N, float2 *__restrict__ hyz) {
    int H = *n_hits;
    if (H > cap_hits) H = cap_hits;
    for (int j = blockIdx.x * TPC_BLOCK + threadIdx.x; j < H; j += gridDim.x * TPC_BLOCK) {
        const int32_t id = hits[j];
        hyz[j] = (uint32_t)id < (uint32_t)N ? make_float2(y[id], z[id]) : make_float2(0.f, 0.f);
    }
}

// Deterministic sum of chi2 over successful tracks: fixed partition of the
// seed range into blocks, fixed reduction tree, FP64 accumulation.
__global__ void __launch_bounds__(TPC_BLOCK)
chi2_partial(const int32_t *__restrict__ n_seeds, int32_t cap_seeds, const float *__restrict__ chi2,
             const int32_t *__restrict__ status, double *__restrict__ part) {
    __shared__ double sh[TPC_BLOCK];
    int T = *n_seeds;
    if (T > cap_seeds) T = cap_seeds;
    const int i = blockIdx.x * TPC_BLOCK + threadIdx.x;
    double v = (i < T && status[i] == TPC_FIT_OK) ? (double)chi2[i] : 0.0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = TPC_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(TPC_BLOCK)
chi2_final(const double *__restrict__ part, int32_t nparts, float *__restrict__ loss) {
    __shared__ double sh[TPC_BLOCK];
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += TPC_BLOCK) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = TPC_BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)sh[0];
}

// Seeds in descending length order (the order within a length is
// immaterial: every seed's fit is its own), so that the lanes of a
// wavefront filter about as many hits each.  Counted per workgroup in LDS
// and added to the global histogram bin by bin; the workgroup then reserves
// one range per length and places its seeds there.
__device__ inline int len_bin(const int32_t *offsets, int i) {
    const int n = offsets[i + 1] - offsets[i];
    return n < TPC_MAX_ROWS ? (n > 0 ? n : 0) : TPC_MAX_ROWS;
}

__global__ void __launch_bounds__(TPC_BLOCK)
fit_order_count(const int32_t *__restrict__ n_seeds, int32_t cap, const int32_t *__restrict__ offsets,
                int32_t *__restrict__ hist, int32_t *__restrict__ cur) {
    __shared__ int lh[TPC_MAX_ROWS + 1];
    for (int b = threadIdx.x; b <= TPC_MAX_ROWS; b += TPC_BLOCK) lh[b] = 0;
    __syncthreads();
    const int T = *n_seeds < cap ? *n_seeds : cap;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        atomicAdd(&lh[len_bin(offsets, i)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b <= TPC_MAX_ROWS; b += TPC_BLOCK)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

__global__ void fit_order_clear(int32_t *__restrict__ hist, int32_t *__restrict__ cur) {
    for (int b = threadIdx.x; b <= TPC_MAX_ROWS; b += blockDim.x) {
        hist[b] = 0;
        cur[b] = 0;
    }
}

// Bin starts in descending length order, and the number of seeds.
__global__ void __launch_bounds__(TPC_WAVE)
fit_order_starts(int32_t *__restrict__ hist, int32_t *__restrict__ n_order) {
    len_starts_wave(hist, n_order);
}

__global__ void __launch_bounds__(TPC_BLOCK)
fit_order_place(const int32_t *__restrict__ n_seeds, int32_t cap, const int32_t *__restrict__ offsets,
                const int32_t *__restrict__ start, int32_t *__restrict__ cur, int32_t *__restrict__ order) {
    __shared__ int lh[TPC_MAX_ROWS + 1], lb[TPC_MAX_ROWS + 1];
    for (int b = threadIdx.x; b <= TPC_MAX_ROWS; b += TPC_BLOCK) lh[b] = 0;
    __syncthreads();
    const int T = *n_seeds < cap ? *n_seeds : cap;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        atomicAdd(&lh[len_bin(offsets, i)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b <= TPC_MAX_ROWS; b += TPC_BLOCK) {
        const int c = lh[b];
        lb[b] = c ? start[b] + atomicAdd(&cur[b], c) : 0;
        lh[b] = 0;
    }
    __syncthreads();
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        const int b = len_bin(offsets, i);
        const int slot = lb[b] + atomicAdd(&lh[b], 1);
        if (slot < T) order[slot] = i;
    }
}

}  // namespace

// The length order of the seeds into ord (workspace); sets A.order.
static void launch_fit_order(FitArgs &A, const FitOrderWs &ord, hipStream_t st) {
    int blocks = (A.cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    hipLaunchKernelGGL(fit_order_clear, dim3(1), dim3(TPC_BLOCK), 0, st, ord.hist, ord.cur);
    hipLaunchKernelGGL(fit_order_count, dim3(blocks), dim3(TPC_BLOCK), 0, st, A.n_seeds, A.cap_seeds, A.offsets,
                       ord.hist, ord.cur);
    hipLaunchKernelGGL(fit_order_starts, dim3(1), dim3(TPC_WAVE), 0, st, ord.hist, ord.n);
    hipLaunchKernelGGL(fit_order_place, dim3(blocks), dim3(TPC_BLOCK), 0, st, A.n_seeds, A.cap_seeds, A.offsets,
                       ord.hist, ord.cur, ord.order);
    A.order = ord.order;
    A.n_order = ord.n;
}

FitArgs make_fit_args(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                      const float *map) {
    const tpc_config &c = ctx->cfg;
    FitArgs A;
    A.offsets = sd->offsets;
    A.hits = sd->hits;
    A.sector = sd->sector;
    A.first_row = sd->first_row;
    A.n_seeds = sd->n_seeds;
    A.cap_seeds = sd->cap_seeds;
    A.cap_hits = sd->cap_hits;
    A.y = fr->y;
    A.z = fr->z;
    A.row_x = ctx->d_row_x;
    A.map = map;
    A.n_rows = c.n_rows;
    A.n_sectors = c.n_sectors;
    A.n_clusters = fr->n_clusters;
    A.kbz = -TPC_C_LIGHT * c.bz;
    A.vy = (double)c.sigma_y * (double)c.sigma_y;
    A.vz = (double)c.sigma_z * (double)c.sigma_z;
    A.max_sin = c.max_sin;
    A.var_s = c.var_sin0;
    A.var_t = c.var_tgl0;
    A.var_w = c.var_qpt0;
    A.ckpt = nullptr;
    A.ckpt_rows = c.ckpt_rows;
    A.hyz = nullptr;
    A.out = tpc_tracks{};
    A.order = nullptr;
    A.n_order = nullptr;
    return A;
}

hipError_t launch_gather(const tpc_frames *fr, const tpc_seeds *sd, float2 *hyz, hipStream_t st) {
    int blocks = (sd->cap_hits + TPC_BLOCK - 1) / TPC_BLOCK;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(gather_hits, dim3(blocks), dim3(TPC_BLOCK), 0, st, sd->n_hits, sd->cap_hits,
                       sd->hits, fr->y, fr->z, fr->n_clusters, hyz);
    return hipGetLastError();
}

hipError_t launch_fit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                      const float *map, const tpc_tracks *tr, double *ckpt, void *ws, hipStream_t st) {
    FitArgs A = make_fit_args(ctx, fr, sd, map);
    A.out = *tr;
    A.ckpt = ckpt;
    float2 *hyz;
    FitOrderWs ord;
    fit_ws_layout(ws, sd->cap_seeds, sd->cap_hits, nullptr, &hyz, &ord);
    if (sd->hit_yz) {
        A.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        A.hyz = hyz;
        launch_gather(fr, sd, hyz, st);
    }
    if (sd->cap_seeds >= TPC_FIT_ORDER_MIN) launch_fit_order(A, ord, st);
    return launch_fit_args(A, st, A.order != nullptr, 0, 0);
}

// Launch shape of the fit: workgroups of `block` threads (0: TPC_BLOCK) and
// about `spt` seeds per thread (0: one) over the seed capacity.
hipError_t launch_fit_args(const FitArgs &A, hipStream_t st, bool ordered, int block, int spt) {
    const int b = block > 0 ? block : TPC_BLOCK;
    const int64_t per = (int64_t)b * (spt > 0 ? spt : 1);
    int64_t blocks = ((int64_t)A.cap_seeds + per - 1) / per;
    const int64_t maxb = (int64_t)8192 * TPC_BLOCK / b;
    if (blocks > maxb) blocks = maxb;
    if (blocks < 1) blocks = 1;
    if (ordered)
        hipLaunchKernelGGL(fit_tracks_ordered, dim3((unsigned)blocks), dim3(b), 0, st, A);
    else
        hipLaunchKernelGGL(fit_tracks, dim3((unsigned)blocks), dim3(b), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_fit_shaped(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                             const tpc_tracks *tr, void *ws, int block, int spt, hipStream_t st) {
    FitArgs A = make_fit_args(ctx, fr, sd, nullptr);
    A.out = *tr;
    A.ckpt = nullptr;
    float2 *hyz;
    FitOrderWs ord;
    fit_ws_layout(ws, sd->cap_seeds, sd->cap_hits, nullptr, &hyz, &ord);
    if (sd->hit_yz) {
        A.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        A.hyz = hyz;
        launch_gather(fr, sd, hyz, st);
    }
    if (sd->cap_seeds >= TPC_FIT_ORDER_MIN) launch_fit_order(A, ord, st);
    return launch_fit_args(A, st, A.order != nullptr, block, spt);
}

size_t chi2_ws_layout(void *ws, int64_t cap_seeds, double **part) {
    WsCarver w(ws);
    const int64_t nb = (cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    double *p = w.take<double>(nb > 0 ? nb : 1);
    if (part) *part = p;
    return (w.off + 255) & ~size_t(255);
}

// Fit workspace: the chi2 partials, the seed-ordered hit coordinates, then
// the length order of the seeds.
size_t fit_ws_layout(void *ws, int64_t cap_seeds, int64_t cap_hits, double **part, float2 **hyz,
                     FitOrderWs *ord) {
    const size_t a = chi2_ws_layout(ws, cap_seeds, part);
    WsCarver w(ws);
    w.off = a;
    float2 *h = w.take<float2>(cap_hits > 0 ? cap_hits : 1);
    if (hyz) *hyz = h;
    int32_t *o = w.take<int32_t>(cap_seeds > 0 ? cap_seeds : 1);
    int32_t *hi = w.take<int32_t>(TPC_MAX_ROWS + 1);
    int32_t *cu = w.take<int32_t>(TPC_MAX_ROWS + 1);
    int32_t *n = w.take<int32_t>(1);
    if (ord) *ord = FitOrderWs{o, hi, cu, n};
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_chi2_sum(const tpc_seeds *sd, const tpc_tracks *tr, float *loss, void *ws,
                           hipStream_t st) {
    double *part;
    chi2_ws_layout(ws, sd->cap_seeds, &part);
    int nb = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(chi2_partial, dim3(nb), dim3(TPC_BLOCK), 0, st, sd->n_seeds, sd->cap_seeds,
                       tr->chi2, tr->status, part);
    hipLaunchKernelGGL(chi2_final, dim3(1), dim3(TPC_BLOCK), 0, st, part, nb, loss);
    return hipGetLastError();
}
