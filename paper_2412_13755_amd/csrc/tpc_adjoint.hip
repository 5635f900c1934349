// Adjoint of the summed fit chi2 with respect to the per-(sector, row)
// cluster correction map (gfx950).
//
// L(M) = sum over successfully fitted seeds of chi2, with every cluster of
// (sector s, row r) corrected by -M[s][r]; dL/dM[s][r] = -(sum of dL/dm over
// the hits of (s, r)), scaled by the caller's upstream gradient dloss.
//
//  adj_tracks   one thread per seed, reverse mode by hand: for each segment of
//               ckpt_rows filter steps, from the innermost backwards, restart
//               from the forward checkpoint, recompute the segment storing the
//               filter state before every step in a per-thread tape (global
//               memory, laid out so a wavefront's accesses are contiguous),
//               then run the step adjoints over it; finally the three-point
//               start.  Writes dL/dm per seed hit.
//  adj_partial  deterministic per-(frame, sector) sums per row: seeds of one
//               (frame, sector) are contiguous (seeds are ordered by their
//               first cluster id); each workgroup sums fixed chunks of them in
//               seed order, one thread per row
//  adj_final    fixed-order sum of the partials, times -dloss
#include "tpc_fit_common.hpp"

namespace {

struct AdjArgs {
    FitArgs F;
    const int32_t *status;
    const double *ckpt;
    float2 *g;          // [cap_hits] dL/d(my, mz) per seed hit
    double *tape;       // [threads / 64][K][TPC_CKPT_WORDS][64]
    int32_t nthreads;
};

// Two wavefronts per SIMD (256 registers per lane, a few spilled): the
// step adjoint's live set is near 300 registers, and one wavefront per SIMD
// leaves its latency exposed.
__global__ void __launch_bounds__(TPC_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
adj_tracks(AdjArgs A) {
    __shared__ float xs[TPC_MAX_ROWS];
    const FitArgs &F = A.F;
    for (int r = threadIdx.x; r < F.n_rows; r += TPC_BLOCK) xs[r] = F.row_x[r];
    __syncthreads();
    int T = *F.n_seeds;
    if (T > F.cap_seeds) T = F.cap_seeds;
    const int gt = blockIdx.x * TPC_BLOCK + threadIdx.x;
    const int K = F.ckpt_rows;
    // this thread's tape: word q of step s at tp[(s * TPC_CKPT_WORDS + q) * 64],
    // so the 64 lanes of a wavefront touch one contiguous 512-byte run
    double *tp = A.tape + (size_t)(gt / TPC_WAVE) * K * TPC_CKPT_WORDS * TPC_WAVE + (gt & (TPC_WAVE - 1));
    for (int i = gt; i < T; i += A.nthreads) adj_one(F, A.status, A.ckpt, A.g, i, xs, tp, TPC_WAVE);
}

// key of seed i: frame * n_sectors + sector (non-decreasing over seeds)
__device__ inline int seed_key(const int32_t *frame, const int32_t *sector, int n_sectors, int i) {
    return frame[i] * n_sectors + sector[i];
}

__device__ inline int lower_bound_key(const int32_t *frame, const int32_t *sector, int n_sectors,
                                      int T, int key) {
    int lo = 0, hi = T;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (seed_key(frame, sector, n_sectors, mid) < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(TPC_BLOCK)
adj_partial(const int32_t *__restrict__ n_seeds, int32_t cap_seeds,
            const int32_t *__restrict__ offsets, const int32_t *__restrict__ first_row,
            const int32_t *__restrict__ frame, const int32_t *__restrict__ sector,
            int32_t n_sectors, int32_t n_rows, const float2 *__restrict__ g,
            float2 *__restrict__ partial) {
    __shared__ int so[TPC_BLOCK], sn[TPC_BLOCK], sr[TPC_BLOCK];
    __shared__ int range[2];
    const int fs = blockIdx.x, gsub = blockIdx.y, G = gridDim.y;
    const int r = threadIdx.x;
    if (threadIdx.x == 0) {
        int T = *n_seeds;
        if (T > cap_seeds) T = cap_seeds;
        range[0] = lower_bound_key(frame, sector, n_sectors, T, fs);
        range[1] = lower_bound_key(frame, sector, n_sectors, T, fs + 1);
    }
    __syncthreads();
    const int lo = range[0], hi = range[1];
    float ay = 0.f, az = 0.f;
    for (int c0 = lo + gsub * TPC_BLOCK; c0 < hi; c0 += G * TPC_BLOCK) {
        const int i = c0 + threadIdx.x;
        if (i < hi) {
            so[threadIdx.x] = offsets[i];
            sn[threadIdx.x] = offsets[i + 1] - offsets[i];
            sr[threadIdx.x] = first_row[i];
        }
        __syncthreads();
        const int cnt = hi - c0 < TPC_BLOCK ? hi - c0 : TPC_BLOCK;
        // a frame-sector's seeds come in non-decreasing first row (seed
        // order is first-cluster id order), so none after the first seed
        // starting above row r reaches r
        for (int q = 0; q < cnt; ++q) {
            if (sr[q] > r) break;
            const int k = r - sr[q];
            // seeds that fail the fit's sanity checks were never written
            const bool sane = sn[q] >= 3 && sr[q] >= 0 && sr[q] + sn[q] <= n_rows && so[q] >= 0;
            if (sane && k >= 0 && k < sn[q]) {
                const float2 v = g[so[q] + k];
                ay += v.x;
                az += v.y;
            }
        }
        __syncthreads();
    }
    if (r < n_rows) partial[((size_t)fs * G + gsub) * n_rows + r] = make_float2(ay, az);
}

__global__ void __launch_bounds__(TPC_BLOCK)
adj_final(const float2 *__restrict__ partial, int32_t n_frames, int32_t n_sectors, int32_t n_rows,
          int32_t G, const float *__restrict__ dloss, float *__restrict__ grad) {
    const int idx = blockIdx.x * TPC_BLOCK + threadIdx.x;
    if (idx >= n_sectors * n_rows) return;
    const int s = idx / n_rows, r = idx % n_rows;
    double ay = 0.0, az = 0.0;
    for (int f = 0; f < n_frames; ++f)
        for (int q = 0; q < G; ++q) {
            const float2 v = partial[((size_t)(f * n_sectors + s) * G + q) * n_rows + r];
            ay += v.x;
            az += v.y;
        }
    const double d = dloss ? (double)*dloss : 1.0;
    grad[(size_t)idx * 2] = (float)(-d * ay);
    grad[(size_t)idx * 2 + 1] = (float)(-d * az);
}

}  // namespace

#define TPC_ADJ_MAX_BLOCKS 512     // persistent grid: 131072 threads, 8 waves per CU
// Workgroups per (frame, sector) in the row sums: enough for about 4096
// workgroups in all, at most 64 (each sums a fixed share of the seeds, so
// the result stays bit-reproducible).
static int adj_groups(int64_t n_fs) {
    int64_t g = n_fs > 0 ? 4096 / n_fs : 1;
    return (int)(g < 1 ? 1 : (g > 64 ? 64 : g));
}

static int adj_blocks(int32_t cap_seeds) {
    int b = (cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (b > TPC_ADJ_MAX_BLOCKS) b = TPC_ADJ_MAX_BLOCKS;
    return b < 1 ? 1 : b;
}

size_t adj_ws_layout(void *ws, int64_t cap_hits, int64_t cap_seeds, int64_t n_fs, int32_t n_rows,
                     int32_t K, float2 **g, double **tape, float2 **partial, float2 **hyz) {
    WsCarver w(ws);
    float2 *pg = w.take<float2>(cap_hits > 0 ? cap_hits : 1);
    const int64_t nthreads = (int64_t)adj_blocks((int32_t)(cap_seeds < 0x7fffffff ? cap_seeds : 0x7fffffff)) * TPC_BLOCK;
    double *pt = w.take<double>(nthreads * K * TPC_CKPT_WORDS);
    float2 *pp = w.take<float2>(n_fs * adj_groups(n_fs) * n_rows);
    float2 *ph = w.take<float2>(cap_hits > 0 ? cap_hits : 1);
    if (hyz) *hyz = ph;
    if (g) *g = pg;
    if (tape) *tape = pt;
    if (partial) *partial = pp;
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_adjoint(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                          const float *map, const tpc_tracks *tr, const double *ckpt,
                          const float *dloss, float *grad_map, void *ws, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    const int64_t n_fs = (int64_t)fr->n_frames * c.n_sectors;
    AdjArgs A;
    A.F = make_fit_args(ctx, fr, sd, map);
    A.status = tr->status;
    A.ckpt = ckpt;
    float2 *partial;
    float2 *hyz;
    adj_ws_layout(ws, sd->cap_hits, sd->cap_seeds, n_fs, c.n_rows, c.ckpt_rows, &A.g, &A.tape, &partial, &hyz);
    if (sd->hit_yz) {
        A.F.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        A.F.hyz = hyz;
        launch_gather(fr, sd, hyz, st);
    }
    const int blocks = adj_blocks(sd->cap_seeds);
    A.nthreads = blocks * TPC_BLOCK;
    hipLaunchKernelGGL(adj_tracks, dim3(blocks), dim3(TPC_BLOCK), 0, st, A);
    const int groups = adj_groups(n_fs);
    hipLaunchKernelGGL(adj_partial, dim3((unsigned)n_fs, groups), dim3(TPC_BLOCK), 0, st,
                       sd->n_seeds, sd->cap_seeds, sd->offsets, sd->first_row, sd->frame,
                       sd->sector, c.n_sectors, c.n_rows, A.g, partial);
    const int nout = c.n_sectors * c.n_rows;
    hipLaunchKernelGGL(adj_final, dim3((nout + TPC_BLOCK - 1) / TPC_BLOCK), dim3(TPC_BLOCK), 0, st,
                       partial, fr->n_frames, c.n_sectors, c.n_rows, groups, dloss, grad_map);
    return hipGetLastError();
}
