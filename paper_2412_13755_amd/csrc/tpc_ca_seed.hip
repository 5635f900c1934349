// Seeding stage kernels: one workgroup per (frame, sector, row) segment for
// every step but the segment scan; the per-segment work is in
// tpc_ca_device.hpp.
#include "tpc_ca_device.hpp"

namespace {

using namespace tpc_ca;

__global__ void __launch_bounds__(TPC_BLOCK)
ca_links(int32_t N, const int32_t *off, const int32_t *up, const int32_t *dn, CaWs ws) {
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    ca_links_seg(seg, N, off, up, dn, ws);
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_block(int32_t n_rows, const int32_t *off, CaWs ws) {
    __shared__ int32_t W[TPC_CA_CAP];
    ca_block_item(xcd_item(blockIdx.x, gridDim.x), n_rows, off, ws, W);
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_tops(int32_t N, const int32_t *off, const int32_t *up, const int32_t *dn, int32_t min_hits,
        int32_t n_rows, CaWs ws) {
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    ca_tops_seg(seg, N, off, up, dn, min_hits, n_rows, ws);
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_firsts(int32_t N, const int32_t *off, const int32_t *up, const int32_t *dn, int32_t min_hits, CaWs ws) {
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    ca_firsts_seg(seg, N, off, up, dn, min_hits, ws);
}

// Single workgroup: exclusive scan of the per-segment counts, chunk by chunk.
__global__ void __launch_bounds__(1024)
ca_scan(int32_t NR, CaWs ws, int32_t *__restrict__ n_seeds, int32_t *__restrict__ n_hits,
        int32_t cap_seeds, int32_t cap_hits, int32_t *__restrict__ offsets,
        int32_t *__restrict__ dev_status) {
    __shared__ int shc[1024 / TPC_WAVE], shh[1024 / TPC_WAVE];
    __shared__ int carry_c, carry_h;
    const int tid = threadIdx.x, lane = tid & (TPC_WAVE - 1), wid = tid / TPC_WAVE;
    if (tid == 0) { carry_c = 0; carry_h = 0; }
    __syncthreads();
    for (int base = 0; base < NR; base += 1024) {
        int i = base + tid;
        int vc = i < NR ? ws.segcnt[i] : 0;
        int vh = i < NR ? ws.seghits[i] : 0;
        int ic = wave_inclusive_scan(vc), ih = wave_inclusive_scan(vh);
        if (lane == TPC_WAVE - 1) { shc[wid] = ic; shh[wid] = ih; }
        __syncthreads();
        int bc = 0, bh = 0, tc = 0, th = 0;
        for (int w = 0; w < 1024 / TPC_WAVE; ++w) {
            bc += w < wid ? shc[w] : 0;
            bh += w < wid ? shh[w] : 0;
            tc += shc[w];
            th += shh[w];
        }
        int cc = carry_c, ch = carry_h;
        if (i < NR) {
            ws.segbs[i] = cc + bc + ic - vc;
            ws.segbh[i] = ch + bh + ih - vh;
        }
        __syncthreads();
        if (tid == 0) { carry_c = cc + tc; carry_h = ch + th; }
        __syncthreads();
    }
    if (tid == 0) {
        int ns = carry_c, nh = carry_h;
        *n_seeds = ns;
        *n_hits = nh;
        bool ok = ns <= cap_seeds && nh <= cap_hits;
        *dev_status = ok ? TPC_OK : TPC_ERR_CAPACITY;
        if (ns <= cap_seeds) offsets[ns] = ok ? nh : 0;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_place(int32_t N, const int32_t *off, const int32_t *up, const int32_t *dn, const float *y, const float *z,
         int32_t n_sectors, int32_t n_rows, int32_t cap_seeds, int32_t cap_hits, tpc_seeds sd, CaWs ws) {
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    ca_place_seg(seg, N, off, up, dn, y, z, n_sectors, n_rows, cap_seeds, cap_hits, sd, ws);
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_members(int32_t N, const int32_t *off, const int32_t *up, const int32_t *dn, const float *y,
           const float *z, int32_t cap_hits, tpc_seeds sd, CaWs ws) {
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    ca_members_seg(seg, N, off, up, dn, y, z, cap_hits, sd, ws);
}

}  // namespace


hipError_t launch_ca_seed(const tpc_context *ctx, const tpc_frames *fr, const int32_t *up,
                          const int32_t *dn, const tpc_seeds *sd, int32_t *dev_status,
                          const CaWs &ws, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    const int NR = fr->n_frames * c.n_sectors * c.n_rows;
    const int32_t *off = fr->row_offsets;
    const int32_t N = fr->n_clusters;
    hipLaunchKernelGGL(ca_links, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, ws);
    const int NB = fr->n_frames * c.n_sectors * ca_blocks_per_sector(c.n_rows);
    hipLaunchKernelGGL(ca_block, dim3(NB), dim3(TPC_BLOCK), 0, st, c.n_rows, off, ws);
    hipLaunchKernelGGL(ca_tops, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, c.min_hits, c.n_rows, ws);
    hipLaunchKernelGGL(ca_firsts, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, c.min_hits, ws);
    hipLaunchKernelGGL(ca_scan, dim3(1), dim3(1024), 0, st, NR, ws, sd->n_seeds, sd->n_hits,
                       sd->cap_seeds, sd->cap_hits, sd->offsets, dev_status);
    hipLaunchKernelGGL(ca_place, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, fr->y, fr->z,
                       c.n_sectors, c.n_rows, sd->cap_seeds, sd->cap_hits, *sd, ws);
    hipLaunchKernelGGL(ca_members, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, fr->y, fr->z,
                       sd->cap_hits, *sd, ws);
    return hipGetLastError();
}

size_t ca_ws_layout(void *ws, int64_t N, int64_t NR, CaWs *out) {
    WsCarver w(ws);
    CaWs l;
    l.claim = w.take<unsigned long long>(N);
    l.pack = w.take<unsigned long long>(N);
    l.dlk = w.take<int32_t>(N);
    l.core = w.take<int32_t>(N);
    l.ctop = w.take<int32_t>(N);
    l.memb = w.take<int32_t>(N);
    l.mpos = w.take<int32_t>(N);
    l.fbot = w.take<int32_t>(N);
    l.flen = w.take<int32_t>(N);
    l.choff = w.take<int32_t>(N);
    l.segcnt = w.take<int32_t>(NR);
    l.seghits = w.take<int32_t>(NR);
    l.segbs = w.take<int32_t>(NR);
    l.segbh = w.take<int32_t>(NR);
    if (out) *out = l;
    return (w.off + 255) & ~size_t(255);
}
