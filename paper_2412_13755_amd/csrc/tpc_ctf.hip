// Track-model residual transform of a frame's clusters into flat integer
// arrays, the input of the entropy coder (gfx950).
//
//  ct_own_init     owner of every cluster := none
//  ct_own          wavefront per kept track: 32-bit atomicMin of the track
//                  index on each of its clusters (lowest index owns)
//  ct_count        wavefront per track: its own clusters, counted by ballot
//  ct_tsum/tscan/tapply  prefixes of kept tracks, row steps and second
//                  differences over the tracks (workgroup sums, their scan,
//                  each workgroup's scan)
//  ct_free         workgroup per segment: free clusters compacted in id order
//                  (block scan), their split quantised values; the segment's
//                  count
//  ct_scan_segs    one workgroup: prefix of free clusters over segments (run
//                  between two ct_free passes: count, then emit)
//  ct_emit         workgroup per kept track: its own clusters compacted in row
//                  order (block scan into LDS), then each thread writes the
//                  row step and residuals of one cluster; the track record
#include "tpc_internal.hpp"

namespace {

struct CtArgs {
    const int32_t *row_offsets;
    const float *y, *z;
    int32_t N, NR, R, S;
    const int32_t *n_seeds;
    int32_t cap_seeds;
    const int32_t *frame, *sector, *rows, *status;
    float iy, iz;                 // 1 / quantisation step, single precision
    int32_t *own;                 // [N]
    int32_t *m;                   // [cap_seeds] own clusters of each kept track
    int32_t *kp, *dp, *rp;        // [cap_seeds + 1] prefixes: kept, row steps, residuals
    int32_t *fp;                  // [NR + 1] prefix of free clusters
    int32_t *bsum;                // [3 per workgroup of tracks] sums, then their prefixes
    tpc_ctf_arrays out;
};

__device__ inline int32_t quant(float v, float inv) {
    const float s = v * inv;
    if (!(s > -1073741824.0f && s < 1073741824.0f)) return 0;
    return (int32_t)rintf(s);
}

__device__ inline int n_tracks(const CtArgs &A) {
    const int T = *A.n_seeds;
    return T < A.cap_seeds ? T : A.cap_seeds;
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_own_init(CtArgs A) {
    for (int c = blockIdx.x * TPC_BLOCK + threadIdx.x; c < A.N; c += gridDim.x * TPC_BLOCK) A.own[c] = 0x7fffffff;
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_own(CtArgs A) {
    const int T = n_tracks(A);
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int W = gridDim.x * (TPC_BLOCK / TPC_WAVE);
    for (int t = blockIdx.x * (TPC_BLOCK / TPC_WAVE) + threadIdx.x / TPC_WAVE; t < T; t += W) {
        if (A.status[t] != TPC_FIT_OK) continue;
        const int32_t *rw = A.rows + (size_t)t * A.R;
        for (int r = lane; r < A.R; r += TPC_WAVE) {
            const int c = rw[r];
            if ((uint32_t)c < (uint32_t)A.N) atomicMin(&A.own[c], t);
        }
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_count(CtArgs A) {
    const int T = n_tracks(A);
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int W = gridDim.x * (TPC_BLOCK / TPC_WAVE);
    for (int t = blockIdx.x * (TPC_BLOCK / TPC_WAVE) + threadIdx.x / TPC_WAVE; t < T; t += W) {
        int cnt = 0;
        if (A.status[t] == TPC_FIT_OK) {
            const int32_t *rw = A.rows + (size_t)t * A.R;
            for (int r0 = 0; r0 < A.R; r0 += TPC_WAVE) {
                const int r = r0 + lane;
                const int c = r < A.R ? rw[r] : -1;
                cnt += __popcll(__ballot((uint32_t)c < (uint32_t)A.N && A.own[c] == t));
            }
        }
        if (lane == 0) A.m[t] = cnt;
    }
}

// Exclusive scans of three per-track counts (kept, row steps, residuals):
// per-workgroup sums, one workgroup over those, then each workgroup's scan.
__device__ inline void track_vals(const CtArgs &A, int t, int T, int v[3]) {
    const bool kept = t < T && A.status[t] == TPC_FIT_OK;
    const int mt = kept ? A.m[t] : 0;
    v[0] = kept ? 1 : 0;
    v[1] = mt > 1 ? mt - 1 : 0;
    v[2] = mt > 2 ? mt - 2 : 0;
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_tsum(CtArgs A) {
    __shared__ int sh[3][TPC_BLOCK / TPC_WAVE];
    const int T = n_tracks(A);
    if ((int)blockIdx.x * TPC_BLOCK >= T) return;
    int v[3], tot[3];
    track_vals(A, blockIdx.x * TPC_BLOCK + threadIdx.x, T, v);
#pragma unroll
    for (int k = 0; k < 3; ++k) block_exclusive_scan(v[k], sh[k], &tot[k]);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) A.bsum[blockIdx.x * 3 + k] = tot[k];
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_tscan(CtArgs A) {
    __shared__ int sh[3][TPC_BLOCK / TPC_WAVE];
    const int T = n_tracks(A);
    const int nb = (T + TPC_BLOCK - 1) / TPC_BLOCK;
    int c[3] = {0, 0, 0};
    for (int b0 = 0; b0 < nb; b0 += TPC_BLOCK) {
        const int b = b0 + threadIdx.x;
        int tot[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int v = b < nb ? A.bsum[b * 3 + k] : 0;
            const int ex = block_exclusive_scan(v, sh[k], &tot[k]);
            if (b < nb) A.bsum[b * 3 + k] = c[k] + ex;
            c[k] += tot[k];
        }
    }
    if (threadIdx.x == 0) {
        A.kp[T] = c[0];
        A.dp[T] = c[1];
        A.rp[T] = c[2];
        for (int k = 0; k < 9; ++k) A.out.counts[k] = c[0];
        A.out.counts[9] = c[1];
        A.out.counts[10] = c[2];
        A.out.counts[11] = c[2];
        A.out.counts[12] = A.NR;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_tapply(CtArgs A) {
    __shared__ int sh[3][TPC_BLOCK / TPC_WAVE];
    const int T = n_tracks(A);
    if ((int)blockIdx.x * TPC_BLOCK >= T) return;
    const int t = blockIdx.x * TPC_BLOCK + threadIdx.x;
    int v[3], tot[3], ex[3];
    track_vals(A, t, T, v);
#pragma unroll
    for (int k = 0; k < 3; ++k) ex[k] = block_exclusive_scan(v[k], sh[k], &tot[k]);
    if (t < T) {
        A.kp[t] = A.bsum[blockIdx.x * 3] + ex[0];
        A.dp[t] = A.bsum[blockIdx.x * 3 + 1] + ex[1];
        A.rp[t] = A.bsum[blockIdx.x * 3 + 2] + ex[2];
    }
}

// emit == false: count the segment's free clusters into fp[s];
// emit == true: write them at fp[s] (the prefix by then) in id order.
__global__ void __launch_bounds__(TPC_BLOCK) ct_free(CtArgs A, int emit) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int s = xcd_item(blockIdx.x, gridDim.x);
    const int a = A.row_offsets[s], n = A.row_offsets[s + 1] - a;
    int base = emit ? A.fp[s] : 0;
    for (int c0 = 0; c0 < n; c0 += TPC_BLOCK) {
        const int c = a + c0 + threadIdx.x;
        const bool fr = c0 + (int)threadIdx.x < n && A.own[c] == 0x7fffffff;
        int tot;
        const int ex = block_exclusive_scan(fr ? 1 : 0, sh, &tot);
        if (emit && fr) {
            const int32_t qy = quant(A.y[c], A.iy), qz = quant(A.z[c], A.iz);
            const int o = base + ex;
            A.out.free_yh[o] = qy >> 8;
            A.out.free_yl[o] = qy & 255;
            A.out.free_zh[o] = qz >> 8;
            A.out.free_zl[o] = qz & 255;
        }
        base += tot;
    }
    if (threadIdx.x == 0) {
        if (emit) A.out.seg_nfree[s] = base - A.fp[s];
        else A.fp[s] = base;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) ct_scan_segs(CtArgs A) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    int carry = 0;
    for (int b = 0; b < A.NR; b += TPC_BLOCK) {
        const int s = b + threadIdx.x;
        const int v = s < A.NR ? A.fp[s] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, sh, &tot);
        if (s < A.NR) A.fp[s] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        A.fp[A.NR] = carry;
        for (int k = 13; k < 17; ++k) A.out.counts[k] = carry;
    }
}

// Workgroup per kept track (TPC_BLOCK >= n_rows threads, thread r on row r):
// its own clusters compacted in row order by a block scan into LDS, then
// thread k writes what cluster k contributes.
__global__ void __launch_bounds__(TPC_BLOCK) ct_emit(CtArgs A) {
    __shared__ int sy[TPC_MAX_ROWS], sz[TPC_MAX_ROWS], sr[TPC_MAX_ROWS];
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int T = n_tracks(A);
    for (int t = blockIdx.x; t < T; t += gridDim.x) {
        if (A.status[t] != TPC_FIT_OK) continue;        // uniform over the workgroup
        const int32_t *rw = A.rows + (size_t)t * A.R;
        int m = 0;
        for (int r0 = 0; r0 < A.R; r0 += TPC_BLOCK) {
            const int r = r0 + threadIdx.x;
            const int c = r < A.R ? rw[r] : -1;
            const bool mine = (uint32_t)c < (uint32_t)A.N && A.own[c] == t;
            int tot;
            const int k = m + block_exclusive_scan(mine ? 1 : 0, sh, &tot);
            if (mine) {
                sy[k] = quant(A.y[c], A.iy);
                sz[k] = quant(A.z[c], A.iz);
                sr[k] = r;
            }
            m += tot;
        }
        __syncthreads();
        const int d = A.dp[t], g = A.rp[t];
        for (int k = threadIdx.x; k < m; k += TPC_BLOCK) {
            if (k >= 1) A.out.hit_drow[d + k - 1] = sr[k] - sr[k - 1] - 1;
            if (k >= 2) {
                A.out.hit_ry[g + k - 2] = sy[k] - 2 * sy[k - 1] + sy[k - 2];
                A.out.hit_rz[g + k - 2] = sz[k] - 2 * sz[k - 1] + sz[k - 2];
            }
        }
        if (threadIdx.x == 0) {
            const int k = A.kp[t];
            const int qy0 = m ? sy[0] : 0, qz0 = m ? sz[0] : 0;
            A.out.trk_seg[k] = A.frame[t] * A.S + A.sector[t];
            A.out.trk_n[k] = m;
            A.out.trk_row0[k] = m ? sr[0] : 0;
            A.out.trk_y0h[k] = qy0 >> 8;
            A.out.trk_y0l[k] = qy0 & 255;
            A.out.trk_z0h[k] = qz0 >> 8;
            A.out.trk_z0l[k] = qz0 & 255;
            A.out.trk_dy1[k] = m >= 2 ? sy[1] - qy0 : 0;
            A.out.trk_dz1[k] = m >= 2 ? sz[1] - qz0 : 0;
        }
        __syncthreads();
    }
}

int grid_for(int64_t items) {
    int64_t b = (items + TPC_BLOCK - 1) / TPC_BLOCK;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

size_t ctf_ws_layout(void *ws, int64_t N, int64_t NR, int64_t cap_seeds, void *out) {
    WsCarver w(ws);
    int32_t *own = w.take<int32_t>(N > 0 ? N : 1);
    int32_t *m = w.take<int32_t>(cap_seeds > 0 ? cap_seeds : 1);
    int32_t *kp = w.take<int32_t>(cap_seeds + 1);
    int32_t *dp = w.take<int32_t>(cap_seeds + 1);
    int32_t *rp = w.take<int32_t>(cap_seeds + 1);
    int32_t *fp = w.take<int32_t>(NR + 1);
    int32_t *bs = w.take<int32_t>(3 * ((cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK + 1));
    if (out) {
        int32_t **p = static_cast<int32_t **>(out);
        p[0] = own; p[1] = m; p[2] = kp; p[3] = dp; p[4] = rp; p[5] = fp; p[6] = bs;
    }
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_ctf_build(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                            const int32_t *rows, const tpc_tracks *tr, float qy, float qz,
                            const tpc_ctf_arrays *out, void *ws, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    CtArgs A;
    A.row_offsets = fr->row_offsets;
    A.y = fr->y;
    A.z = fr->z;
    A.N = fr->n_clusters;
    A.NR = fr->n_frames * c.n_sectors * c.n_rows;
    A.R = c.n_rows;
    A.S = c.n_sectors;
    A.n_seeds = sd->n_seeds;
    A.cap_seeds = sd->cap_seeds;
    A.frame = sd->frame;
    A.sector = sd->sector;
    A.rows = rows;
    A.status = tr->status;
    A.iy = 1.0f / qy;
    A.iz = 1.0f / qz;
    int32_t *p[7];
    ctf_ws_layout(ws, A.N, A.NR, A.cap_seeds, p);
    A.own = p[0];
    A.m = p[1];
    A.kp = p[2];
    A.dp = p[3];
    A.rp = p[4];
    A.fp = p[5];
    A.bsum = p[6];
    A.out = *out;
    const int wb = grid_for((int64_t)A.cap_seeds * TPC_WAVE);
    hipLaunchKernelGGL(ct_own_init, dim3(grid_for(A.N)), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_own, dim3(wb), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_count, dim3(wb), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_tsum, dim3((A.cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_tscan, dim3(1), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_tapply, dim3((A.cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_free, dim3(A.NR), dim3(TPC_BLOCK), 0, st, A, 0);
    hipLaunchKernelGGL(ct_scan_segs, dim3(1), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(ct_free, dim3(A.NR), dim3(TPC_BLOCK), 0, st, A, 1);
    hipLaunchKernelGGL(ct_emit, dim3(A.cap_seeds < 32768 ? (A.cap_seeds > 0 ? A.cap_seeds : 1) : 32768),
                       dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}
