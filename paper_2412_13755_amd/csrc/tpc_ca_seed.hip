// Seeding stage kernels: one workgroup per (frame, sector, row) segment for
// every step but the segment scan; the per-segment work is in
// tpc_ca_device.hpp.
#include "tpc_ca_device.hpp"

namespace {

using namespace tpc_ca;

__global__ void __launch_bounds__(1024)
ca_block(int32_t N, int32_t n_rows, const int32_t *off, const int32_t *up, const int32_t *dn, CaWs ws) {
    __shared__ uint32_t W[TPC_CA_CAP];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (ca_block_class(item, n_rows, off) == 1) return;
    ca_block_item(item, N, n_rows, off, up, dn, ws, W);
}

// Blocks too large for the LDS ranking with rows of at most
// TPC_CA_SWEEP_ROW clusters: ranked by a bottom-up row sweep.
__global__ void __launch_bounds__(1024)
ca_block_sweep(int32_t NB, int32_t N, int32_t n_rows, const int32_t *off, const int32_t *up, const int32_t *dn,
               CaWs ws) {
    __shared__ uint32_t P[2 * TPC_CA_SWEEP_ROW];
    for (int it = blockIdx.x; it < NB; it += gridDim.x) {
        const int item = xcd_item(it, NB);
        if (ca_block_class(item, n_rows, off) == 1) ca_sweep_item(item, N, n_rows, off, up, dn, ws, P);
    }
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

// Single workgroup: exclusive scan of n (seed count, hit count) pairs into
// (pre_c, pre_h), totals into *n_seeds / *n_hits with the capacity check.
// Thread t owns the contiguous run [t k, (t+1) k), k = ceil(n / 1024): it
// sums its run, one workgroup scan turns run sums into run starts, and it
// writes the prefixes of its run.  Used on the segments directly when they
// are few, else on the chunk sums of ca_chunk_sums.
__global__ void __launch_bounds__(1024)
ca_scan(int32_t n, const int32_t *cnt, const int32_t *hits, int32_t *pre_c, int32_t *pre_h,
        int32_t *__restrict__ n_seeds,
        int32_t *__restrict__ n_hits, int32_t cap_seeds, int32_t cap_hits, int32_t *__restrict__ offsets,
        int32_t *__restrict__ dev_status) {
    __shared__ int shc[1024 / TPC_WAVE], shh[1024 / TPC_WAVE];
    const int tid = threadIdx.x, lane = tid & (TPC_WAVE - 1), wid = tid / TPC_WAVE;
    const int k = (n + 1023) / 1024;
    const int s0 = tid * k < n ? tid * k : n;
    const int s1 = s0 + k < n ? s0 + k : n;
    int vc = 0, vh = 0;
    for (int s = s0; s < s1; ++s) {
        vc += cnt[s];
        vh += hits[s];
    }
    const int ic = wave_inclusive_scan(vc), ih = wave_inclusive_scan(vh);
    if (lane == TPC_WAVE - 1) { shc[wid] = ic; shh[wid] = ih; }
    __syncthreads();
    int bc = 0, bh = 0, tc = 0, th = 0;
#pragma unroll
    for (int w = 0; w < 1024 / TPC_WAVE; ++w) {
        bc += w < wid ? shc[w] : 0;
        bh += w < wid ? shh[w] : 0;
        tc += shc[w];
        th += shh[w];
    }
    int pc = bc + ic - vc, ph = bh + ih - vh;
    for (int s = s0; s < s1; ++s) {              // in place allowed: read before write
        const int c = cnt[s], h = hits[s];
        pre_c[s] = pc;
        pre_h[s] = ph;
        pc += c;
        ph += h;
    }
    if (tid == 0) {
        *n_seeds = tc;
        *n_hits = th;
        const bool ok = tc <= cap_seeds && th <= cap_hits;
        *dev_status = ok ? TPC_OK : TPC_ERR_CAPACITY;
        if (tc <= cap_seeds) offsets[tc] = ok ? th : 0;
    }
}

// Many segments: sums of chunks of TPC_SCAN_CHUNK segments (one workgroup
// per chunk) ...
__global__ void __launch_bounds__(TPC_BLOCK)
ca_chunk_sums(int32_t NR, CaWs ws) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int ch = blockIdx.x, s0 = ch * TPC_SCAN_CHUNK;
    int vc = 0, vh = 0;
    for (int s = s0 + threadIdx.x; s < s0 + TPC_SCAN_CHUNK && s < NR; s += TPC_BLOCK) {
        vc += ws.segcnt[s];
        vh += ws.seghits[s];
    }
    int tc, th;
    block_exclusive_scan(vc, sh, &tc);
    block_exclusive_scan(vh, sh, &th);
    if (threadIdx.x == 0) { ws.chunk_c[ch] = tc; ws.chunk_h[ch] = th; }
}

// ... and, after ca_scan over the chunk sums, the segment prefixes within
// each chunk (thread t owns segments s0 + 4t .. 4t + 3).
__global__ void __launch_bounds__(TPC_BLOCK)
ca_chunk_prefix(int32_t NR, CaWs ws) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    constexpr int PER = TPC_SCAN_CHUNK / TPC_BLOCK;
    const int ch = blockIdx.x, s0 = ch * TPC_SCAN_CHUNK + threadIdx.x * PER;
    int c[PER], h[PER], vc = 0, vh = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool in = s0 + j < NR;
        c[j] = in ? ws.segcnt[s0 + j] : 0;
        h[j] = in ? ws.seghits[s0 + j] : 0;
        vc += c[j];
        vh += h[j];
    }
    int tc, th;
    int pc = ws.chunk_c[ch] + block_exclusive_scan(vc, sh, &tc);
    int ph = ws.chunk_h[ch] + block_exclusive_scan(vh, sh, &th);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (s0 + j < NR) { ws.segbs[s0 + j] = pc; ws.segbh[s0 + j] = ph; }
        pc += c[j];
        ph += h[j];
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
    const int NB = fr->n_frames * c.n_sectors * ca_blocks_per_sector(c.n_rows);
    hipLaunchKernelGGL(ca_block, dim3(NB), dim3(1024), 0, st, N, c.n_rows, off, up, dn, ws);
    const bool sparse = (int64_t)N < (int64_t)TPC_SPARSE_ROW * fr->n_frames * c.n_sectors * c.n_rows;
    hipLaunchKernelGGL(ca_block_sweep, dim3(sparse && NB > TPC_SPARSE_GRID ? TPC_SPARSE_GRID : NB), dim3(1024), 0,
                       st, NB, N, c.n_rows, off, up, dn, ws);
    hipLaunchKernelGGL(ca_tops, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, c.min_hits, c.n_rows, ws);
    hipLaunchKernelGGL(ca_firsts, dim3(NR), dim3(TPC_BLOCK), 0, st, N, off, up, dn, c.min_hits, ws);
    if (NR <= TPC_SCAN_DIRECT) {
        hipLaunchKernelGGL(ca_scan, dim3(1), dim3(1024), 0, st, NR, ws.segcnt, ws.seghits, ws.segbs,
                           ws.segbh, sd->n_seeds, sd->n_hits, sd->cap_seeds, sd->cap_hits, sd->offsets,
                           dev_status);
    } else {
        const int nch = (NR + TPC_SCAN_CHUNK - 1) / TPC_SCAN_CHUNK;
        hipLaunchKernelGGL(ca_chunk_sums, dim3(nch), dim3(TPC_BLOCK), 0, st, NR, ws);
        hipLaunchKernelGGL(ca_scan, dim3(1), dim3(1024), 0, st, nch, ws.chunk_c, ws.chunk_h, ws.chunk_c,
                           ws.chunk_h, sd->n_seeds, sd->n_hits, sd->cap_seeds, sd->cap_hits, sd->offsets,
                           dev_status);
        hipLaunchKernelGGL(ca_chunk_prefix, dim3(nch), dim3(TPC_BLOCK), 0, st, NR, ws);
    }
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
    l.cc = w.take<int2>(N);
    l.cend = w.take<int32_t>(N);
    l.mrec = w.take<int2>(N);
    l.fbot = w.take<int32_t>(N);
    l.flen = w.take<int32_t>(N);
    l.segcnt = w.take<int32_t>(NR);
    l.seghits = w.take<int32_t>(NR);
    l.segbs = w.take<int32_t>(NR);
    l.segbh = w.take<int32_t>(NR);
    const int64_t nch = (NR + TPC_SCAN_CHUNK - 1) / TPC_SCAN_CHUNK;
    l.chunk_c = w.take<int32_t>(nch > 0 ? nch : 1);
    l.chunk_h = w.take<int32_t>(nch > 0 ? nch : 1);
    if (out) *out = l;
    return (w.off + 255) & ~size_t(255);
}
