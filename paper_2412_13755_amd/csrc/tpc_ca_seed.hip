// Cellular-automaton seeding (gfx950): mutual links -> chains -> end claims
// -> seeds in CSR form, ordered by the global id of their first cluster.
//
// All kernels but the segment scan run one workgroup per (frame, sector,
// row) segment with threads over the segment's clusters, so the pad row of
// a cluster is known without a search.  Integer-only; the result is unique
// (claims resolve with a 64-bit atomicMin on a key that orders by chain
// length, then bottom id; seeds are placed by prefix sums in cluster-id
// order), so it matches the sequential definition exactly.
//
//   ca_chains  bottoms (no kept link down, a kept link up) walk their chain,
//              recording the bottom and position of every member, its length
//              and top; every cluster's claim slot is reset
//   ca_claims  chains of >= min_hits-2 clusters claim their unlinked ends
//   ca_firsts  each seed is recognised at its first cluster (the won bottom
//              end or the bottom itself); per-segment seed and hit counts
//   ca_scan    exclusive prefix over segments, totals, capacity check
//   ca_place   seed records, end clusters, core offsets
//   ca_members every chain member writes itself into its seed
#include "tpc_internal.hpp"

namespace {

// Link helpers.  Ids outside [0, N) read as "no link", so corrupt input can
// never address memory outside the arrays.
__device__ inline int32_t link_up(const int32_t *up, const int32_t *dn, int32_t N, int32_t h) {
    int32_t u = up[h];
    return ((uint32_t)u < (uint32_t)N && dn[u] == h) ? u : -1;
}
__device__ inline int32_t link_dn(const int32_t *up, const int32_t *dn, int32_t N, int32_t h) {
    int32_t d = dn[h];
    return ((uint32_t)d < (uint32_t)N && up[d] == h) ? d : -1;
}
__device__ inline bool linked(const int32_t *up, const int32_t *dn, int32_t N, int32_t h) {
    return link_up(up, dn, N, h) >= 0 || link_dn(up, dn, N, h) >= 0;
}
__device__ inline bool valid_id(int32_t v, int32_t N) { return (uint32_t)v < (uint32_t)N; }
__device__ inline unsigned long long claim_key(int32_t m, int32_t b) {
    return ((unsigned long long)(2147483648u - (uint32_t)m) << 32) | (uint32_t)b;
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_chains(const int32_t *__restrict__ off, const int32_t *__restrict__ up,
          const int32_t *__restrict__ dn, int32_t n_rows, CaWs ws) {
    const int seg = blockIdx.x;
    const int a = off[seg], b = off[seg + 1];
    const int32_t N = off[gridDim.x];
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) {
        ws.claim[h] = ~0ull;
        int32_t u = link_up(up, dn, N, h);
        bool bottom = (u >= 0) && link_dn(up, dn, N, h) < 0;
        if (!bottom) {
            ws.core[h] = 0;
            continue;
        }
        ws.memb[h] = h;
        ws.mpos[h] = 0;
        int32_t cur = h, m = 1;
        // walk: one dependent load pair per step; a chain holds at most one
        // cluster per row, which also bounds the walk on corrupt input
        while (u >= 0 && m < n_rows) {
            cur = u;
            ws.memb[cur] = h;
            ws.mpos[cur] = m;
            ++m;
            u = link_up(up, dn, N, cur);
        }
        ws.core[h] = m;
        ws.ctop[h] = cur;
        ws.choff[h] = -1;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_claims(const int32_t *__restrict__ off, const int32_t *__restrict__ up,
          const int32_t *__restrict__ dn, int32_t min_hits, CaWs ws) {
    const int seg = blockIdx.x;
    const int a = off[seg], b = off[seg + 1];
    const int32_t N = off[gridDim.x];
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) {
        int32_t m = ws.core[h];
        if (m < 2 || m < min_hits - 2) continue;
        unsigned long long key = claim_key(m, h);
        int32_t eb = dn[h], et = up[ws.ctop[h]];
        if (valid_id(eb, N) && !linked(up, dn, N, eb)) atomicMin(&ws.claim[eb], key);
        if (valid_id(et, N) && !linked(up, dn, N, et)) atomicMin(&ws.claim[et], key);
    }
}

// Seed length of the chain with bottom bb (0 if it is no seed).
__device__ inline int32_t seed_len(const int32_t *up, const int32_t *dn, int32_t N, int32_t min_hits,
                                   const CaWs &ws, int32_t bb, int32_t *won_b) {
    int32_t m = ws.core[bb];
    int32_t wb = 0, wt = 0;
    if (m >= min_hits - 2) {
        unsigned long long key = claim_key(m, bb);
        int32_t eb = dn[bb], et = up[ws.ctop[bb]];
        wb = (valid_id(eb, N) && ws.claim[eb] == key);
        wt = (valid_id(et, N) && ws.claim[et] == key);
    }
    *won_b = wb;
    int32_t len = m + wb + wt;
    return len >= min_hits ? len : 0;
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_firsts(const int32_t *__restrict__ off, const int32_t *__restrict__ up,
          const int32_t *__restrict__ dn, int32_t min_hits, CaWs ws) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int seg = blockIdx.x;
    const int a = off[seg], b = off[seg + 1];
    const int32_t N = off[gridDim.x];
    int cnt = 0, hits = 0;
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) {
        int32_t fb = -1, len = 0;
        if (ws.core[h] >= 2) {                       // h is a bottom
            int32_t wb;
            int32_t l = seed_len(up, dn, N, min_hits, ws, h, &wb);
            if (l > 0 && !wb) { fb = h; len = l; }
        } else if (ws.claim[h] != ~0ull) {           // h is a claimed end
            int32_t bb = (int32_t)(ws.claim[h] & 0xffffffffull);
            if (valid_id(bb, N) && dn[bb] == h) {    // claimed as the bottom end of bb
                int32_t wb;
                int32_t l = seed_len(up, dn, N, min_hits, ws, bb, &wb);
                if (l > 0) { fb = bb; len = l; }
            }
        }
        ws.fbot[h] = fb;
        ws.flen[h] = len;
        cnt += fb >= 0;
        hits += len;
    }
    int tc, th;
    block_exclusive_scan(cnt, sh, &tc);
    block_exclusive_scan(hits, sh, &th);
    if (threadIdx.x == 0) {
        ws.segcnt[seg] = tc;
        ws.seghits[seg] = th;
    }
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
ca_place(const int32_t *__restrict__ off, const int32_t *__restrict__ up,
         const int32_t *__restrict__ dn, int32_t n_sectors, int32_t n_rows, int32_t cap_seeds,
         int32_t cap_hits, tpc_seeds sd, CaWs ws) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int seg = blockIdx.x;
    const int a = off[seg], b = off[seg + 1];
    int carry_c = ws.segbs[seg], carry_h = ws.segbh[seg];
    const int frame = seg / (n_sectors * n_rows);
    const int sector = (seg / n_rows) % n_sectors;
    const int row = seg % n_rows;
    for (int base = a; base < b; base += TPC_BLOCK) {
        const int h = base + threadIdx.x;
        int32_t fb = -1, len = 0;
        if (h < b) { fb = ws.fbot[h]; len = ws.flen[h]; }
        int tc, th;
        int pc = block_exclusive_scan(fb >= 0 ? 1 : 0, sh, &tc);
        int ph = block_exclusive_scan(len, sh, &th);
        if (fb >= 0) {
            const int i = carry_c + pc;
            const int o = carry_h + ph;
            if (i < cap_seeds && o + len <= cap_hits) {
                sd.offsets[i] = o;
                sd.frame[i] = frame;
                sd.sector[i] = sector;
                sd.first_row[i] = row;
                const int32_t wb = (h != fb);
                if (wb) sd.hits[o] = h;
                const int32_t m = ws.core[fb];
                if (len > m + wb) sd.hits[o + len - 1] = up[ws.ctop[fb]];
                ws.choff[fb] = o + wb;
            }
        }
        carry_c += tc;
        carry_h += th;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
ca_members(const int32_t *__restrict__ off, const int32_t *__restrict__ up,
           const int32_t *__restrict__ dn, int32_t cap_hits, tpc_seeds sd, CaWs ws) {
    const int seg = blockIdx.x;
    const int a = off[seg], b = off[seg + 1];
    const int32_t N = off[gridDim.x];
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) {
        if (!linked(up, dn, N, h)) continue;
        const int32_t bb = ws.memb[h];
        if (!valid_id(bb, N)) continue;
        const int32_t o = ws.choff[bb], k = ws.mpos[h];
        if (o >= 0 && k >= 0 && k < ws.core[bb] && o + k < cap_hits) sd.hits[o + k] = h;
    }
}

}  // namespace

hipError_t launch_ca_seed(const tpc_context *ctx, const tpc_frames *fr, const int32_t *up,
                          const int32_t *dn, const tpc_seeds *sd, int32_t *dev_status,
                          const CaWs &ws, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    const int NR = fr->n_frames * c.n_sectors * c.n_rows;
    const int32_t *off = fr->row_offsets;
    hipLaunchKernelGGL(ca_chains, dim3(NR), dim3(TPC_BLOCK), 0, st, off, up, dn, c.n_rows, ws);
    hipLaunchKernelGGL(ca_claims, dim3(NR), dim3(TPC_BLOCK), 0, st, off, up, dn, c.min_hits, ws);
    hipLaunchKernelGGL(ca_firsts, dim3(NR), dim3(TPC_BLOCK), 0, st, off, up, dn, c.min_hits, ws);
    hipLaunchKernelGGL(ca_scan, dim3(1), dim3(1024), 0, st, NR, ws, sd->n_seeds, sd->n_hits,
                       sd->cap_seeds, sd->cap_hits, sd->offsets, dev_status);
    hipLaunchKernelGGL(ca_place, dim3(NR), dim3(TPC_BLOCK), 0, st, off, up, dn, c.n_sectors,
                       c.n_rows, sd->cap_seeds, sd->cap_hits, *sd, ws);
    hipLaunchKernelGGL(ca_members, dim3(NR), dim3(TPC_BLOCK), 0, st, off, up, dn, sd->cap_hits, *sd, ws);
    return hipGetLastError();
}

size_t ca_ws_layout(void *ws, int64_t N, int64_t NR, CaWs *out) {
    WsCarver w(ws);
    CaWs l;
    l.claim = w.take<unsigned long long>(N);
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
