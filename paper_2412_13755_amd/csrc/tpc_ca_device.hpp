#pragma once
// Cellular-automaton seeding (gfx950): mutual links -> chains -> end claims
// -> seeds in CSR form, ordered by the global id of their first cluster.
// Per-segment device functions, used by the stage kernels and by the
// persistent kernel.
//
// All kernels but the segment scan run one workgroup per (frame, sector,
// row) segment with threads over the segment's clusters, so the pad row of
// a cluster is known without a search.  Integer-only; the result is unique
// (claims resolve with a 64-bit atomicMin on a key that orders by chain
// length, then bottom id; seeds are placed by prefix sums in cluster-id
// order), so it matches the sequential definition exactly.
//
//   ca_block   per (frame, sector, block of TPC_CA_ROWS rows): kept links
//              of every cluster (resetting its claim and length slots), then
//              pointer jumping in LDS to the lowest chain member inside the
//              block and the distance to it (pack)
//   ca_tops    chain tops and block-local lowest members follow the lowest
//              members down across block edges to the chain bottom (at most
//              one hop per block); a lowest member records its bottom and
//              position, each chain's top records its length and claims the
//              chain's unlinked ends (>= min_hits-2 clusters)
//   ca_firsts  each seed is recognised at its first cluster (the won bottom
//              end or the bottom itself); per-segment seed and hit counts
//   ca_scan    exclusive prefix over segments, totals, capacity check
//   ca_place   seed records, end clusters, core offsets
//   ca_members every chain member writes itself into its seed (bottom and
//              position from its block's lowest member)
#include "tpc_internal.hpp"

namespace tpc_ca {


// Ids outside [0, N) read as "no link", so corrupt input can never address
// memory outside the arrays.
__device__ inline bool valid_id(int32_t v, int32_t N) { return (uint32_t)v < (uint32_t)N; }
// (y, z) of seed hit j into the optional coordinate copy (one 8-byte store)
__device__ inline void put_yz(float *hit_yz, int32_t j, float yv, float zv) {
    reinterpret_cast<float2 *>(hit_yz)[j] = make_float2(yv, zv);
}
__device__ inline unsigned long long claim_key(int32_t m, int32_t b) {
    return ((unsigned long long)(2147483648u - (uint32_t)m) << 32) | (uint32_t)b;
}

// Chain ranking.  dlk[h] is the kept link down of h (or -1); a chain is a
// path of such links, one row per link.  Rows are grouped in blocks of
// TPC_CA_ROWS per (frame, sector); pack[h] holds the lowest member of h's
// chain inside h's block (bits 0-31, global id), how many links down it is
// (bits 32-59), whether that member is the chain's bottom (it keeps no link
// down, bit 61; set by the LDS rankings, so that ca_tops need not look) and
// whether h keeps a link up (bit 62) / down (bit 63).

#ifndef TPC_CA_ROWS
#define TPC_CA_ROWS 16          // rows per ranking block
#endif
#define TPC_CA_CAP 8192         // clusters per block ranked in LDS
#ifndef TPC_CA_ROUNDS
#define TPC_CA_ROUNDS 5         // > log2(TPC_CA_ROWS): links inside a block
#endif
#define TPC_CA_BOT (1ull << 61)
#define TPC_CA_UP (1ull << 62)
#define TPC_CA_DN (1ull << 63)
// LDS word: local node (bits 0-19), distance (20-29), up (30), down (31)
#define TPC_CA_NODE 0xFFFFFu
#define TPC_CA_FLAGS 0xC0000000u

__host__ __device__ inline int ca_blocks_per_sector(int n_rows) {
    return (n_rows + TPC_CA_ROWS - 1) / TPC_CA_ROWS;
}
__device__ inline int32_t pack_node(unsigned long long w) { return (int32_t)(uint32_t)w; }
__device__ inline int32_t pack_dist(unsigned long long w) { return (int32_t)((w >> 32) & 0xFFFFFFFull); }
__device__ inline bool pack_linked(unsigned long long w) { return (w & (TPC_CA_UP | TPC_CA_DN)) != 0; }

// Step 1, block `item` of (frame, sector, row block): the kept links of
// every cluster (its slots for claims and chain length are reset on the
// way), then in-place pointer jumping to the lowest chain
// member inside the block (a word always holds a valid (node, distance)
// pair, so reading a neighbour's word before or after its update in the
// same round is equally correct, and every round at least doubles the span
// of a pointer that has not reached its target).  Blocks of at most
// TPC_CA_CAP clusters jump in LDS (W: TPC_CA_CAP words); larger ones in pack
// itself.  Any workgroup size that is a multiple of 64.  Contains barriers:
// call from the whole workgroup.
__device__ inline void ca_block_item(int item, int32_t N, int32_t n_rows, const int32_t *__restrict__ off,
                                     const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                     const CaWs &ws, uint32_t *W) {
    constexpr int U = 4;                              // clusters per thread with loads in flight
    const int nbs = ca_blocks_per_sector(n_rows);
    const int fs = item / nbs, bb = item % nbs;
    const int r0 = bb * TPC_CA_ROWS;
    const int r1 = r0 + TPC_CA_ROWS < n_rows ? r0 + TPC_CA_ROWS : n_rows;
    const int lo = off[fs * n_rows + r0], hi = off[fs * n_rows + r1];
    const int n = hi - lo, tid = threadIdx.x, T = blockDim.x;
    const bool lds = n <= TPC_CA_CAP;
    for (int k0 = tid; k0 < n; k0 += U * T) {
        int32_t d[U], u[U], bd[U], bu[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = k0 + j * T;
            d[j] = k < n ? dn[lo + k] : -1;
            u[j] = k < n ? up[lo + k] : -1;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            bd[j] = valid_id(d[j], N) ? up[d[j]] : -1;
            bu[j] = valid_id(u[j], N) ? dn[u[j]] : -1;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = k0 + j * T;
            if (k >= n) break;
            const int32_t h = lo + k;
            const bool hd = bd[j] == h, hu = bu[j] == h;
            ws.claim[h] = ~0ull;
            ws.cc[h] = make_int2(0, -1);
            ws.dlk[h] = hd ? d[j] : -1;
            const bool in = hd && d[j] >= lo && d[j] < hi && d[j] != h;
            if (lds) {
                W[k] = (hu ? 0x40000000u : 0u) | (hd ? 0x80000000u : 0u) |
                       (in ? ((1u << 20) | (uint32_t)(d[j] - lo)) : (uint32_t)k);
            } else {
                const unsigned long long w = (hu ? TPC_CA_UP : 0ull) | (hd ? TPC_CA_DN : 0ull) |
                                             (in ? ((1ull << 32) | (uint32_t)d[j]) : (uint32_t)h);
                __hip_atomic_store(&ws.pack[h], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    if (lds) {
        for (int round = 0; round < TPC_CA_ROUNDS; ++round) {
            for (int k0 = tid; k0 < n; k0 += U * T) {
                uint32_t v[U], v2[U];
#pragma unroll
                for (int j = 0; j < U; ++j) v[j] = k0 + j * T < n ? W[k0 + j * T] : (uint32_t)(k0 + j * T);
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const uint32_t p = v[j] & TPC_CA_NODE;
                    v2[j] = (k0 + j * T < n && p != (uint32_t)(k0 + j * T)) ? W[p] : 0u;
                }
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int k = k0 + j * T;
                    const uint32_t p = v[j] & TPC_CA_NODE, q = v2[j] & TPC_CA_NODE;
                    if (k < n && p != (uint32_t)k && q != p) {
                        const uint32_t dist = ((v[j] >> 20) & 0x3FFu) + ((v2[j] >> 20) & 0x3FFu);
                        W[k] = (v[j] & TPC_CA_FLAGS) | ((dist & 0x3FFu) << 20) | q;
                    }
                }
            }
            __syncthreads();
        }
        for (int k = tid; k < n; k += T) {
            const uint32_t v = W[k];
            // the lowest member keeps no link down: it is the chain's bottom
            const bool bot = !(W[v & TPC_CA_NODE] & 0x80000000u);
            ws.pack[lo + k] = ((unsigned long long)(v >> 30) << 62) | (bot ? TPC_CA_BOT : 0ull) |
                              ((unsigned long long)((v >> 20) & 0x3FFu) << 32) |
                              (uint32_t)(lo + (int32_t)(v & TPC_CA_NODE));
        }
        __syncthreads();             // LDS reuse across calls in a persistent loop
        return;
    }
    // large block: the same rounds on the global words (written by this
    // workgroup only, so workgroup-scope accesses suffice)
    for (int round = 0; round < TPC_CA_ROUNDS; ++round) {
        for (int k = lo + tid; k < hi; k += T) {
            const unsigned long long v =
                __hip_atomic_load(&ws.pack[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int32_t p = pack_node(v);
            if (p == k) continue;
            const unsigned long long v2 =
                __hip_atomic_load(&ws.pack[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int32_t q = pack_node(v2);
            if (q != p) {
                const unsigned long long dist = (unsigned long long)(pack_dist(v) + pack_dist(v2));
                __hip_atomic_store(&ws.pack[k], (v & (TPC_CA_UP | TPC_CA_DN)) | (dist << 32) | (uint32_t)q,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
    }
}

// Blocks of more than TPC_CA_CAP clusters whose rows each hold at most
// TPC_CA_SWEEP_ROW clusters are ranked by a sweep over their rows from the
// bottom up instead (ca_sweep_item); larger rows jump in pack.
#define TPC_CA_SWEEP_ROW 20480      // 2 x 20480 words: the whole 160 KB of LDS (a multiple of 1024)

// Which ranking a block uses: 0 jumping in LDS, 1 row sweep, 2 jumping in
// global memory.
__device__ inline int ca_block_class(int item, int32_t n_rows, const int32_t *__restrict__ off) {
    const int nbs = ca_blocks_per_sector(n_rows);
    const int fs = item / nbs, bb = item % nbs;
    const int r0 = bb * TPC_CA_ROWS;
    const int r1 = r0 + TPC_CA_ROWS < n_rows ? r0 + TPC_CA_ROWS : n_rows;
    if (off[fs * n_rows + r1] - off[fs * n_rows + r0] <= TPC_CA_CAP) return 0;
    for (int r = r0; r < r1; ++r)
        if (off[fs * n_rows + r + 1] - off[fs * n_rows + r] > TPC_CA_SWEEP_ROW) return 2;
    return 1;
}

// Step 1 for a block of class 1: the same outputs as ca_block_item, by a
// sweep over the block's rows from the bottom up that keeps the previous
// row in LDS: its up partners (pu) and its words (pw: member - lo in bits
// 0-23, distance in 24-28, the member is the chain's bottom in bit 29, keeps
// a link up in bit 30, down in bit 31).  For
// a cluster h of row r with partner d = dn[h] in row r - 1 the link is kept
// if pu says d's up partner is h; then d keeps its link up (its bit 30 is
// set from here), and, inside the block, h's lowest member and distance are
// d's, one link further.  Partners outside the adjacent rows (links across
// a missing row) are checked in global memory, and the ranking then starts
// at h; ca_tops continues any ranking down through kept links, so the
// bottoms and positions it finds are the same.  A row's words go to pack
// one row later, once the row above has set their up bits, so every global
// access but those of the links across a missing row is coalesced.
// P: 2 x TPC_CA_SWEEP_ROW words.  Contains barriers: call from the whole
// workgroup of TPC_CA_SWEEP_T threads.
#define TPC_CA_SWEEP_T 1024
#define TPC_CA_W_BOT 0x20000000u
#define TPC_CA_W_UP 0x40000000u
#define TPC_CA_W_DN 0x80000000u
__device__ inline void ca_sweep_item(int item, int32_t N, int32_t n_rows, const int32_t *__restrict__ off,
                                     const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                     const CaWs &ws, uint32_t *P) {
    constexpr int J = TPC_CA_SWEEP_ROW / TPC_CA_SWEEP_T;   // clusters of a row per thread
    const int nbs = ca_blocks_per_sector(n_rows);
    const int fs = item / nbs, bb = item % nbs;
    const int r0 = bb * TPC_CA_ROWS;
    const int r1 = r0 + TPC_CA_ROWS < n_rows ? r0 + TPC_CA_ROWS : n_rows;
    const int32_t *ro = off + fs * n_rows;            // row starts of this (frame, sector)
    const int lo = ro[r0];
    const int tid = threadIdx.x;
    uint32_t *pw = P, *pu = P + TPC_CA_SWEEP_ROW;
    // the up partners of the row below the block
    int pa = 0, pb = 0;
    if (r0 > 0) {
        pa = ro[r0 - 1];
        pb = ro[r0];
        for (int k = tid; k < pb - pa; k += TPC_CA_SWEEP_T) pu[k] = (uint32_t)up[pa + k];
    }
    __syncthreads();
    for (int r = r0; r < r1; ++r) {
        const int a = ro[r], n = ro[r + 1] - a;
        const int na = r + 1 < n_rows ? ro[r + 1] : 0, nb = r + 1 < n_rows ? ro[r + 2] : 0;  // row above
        int32_t uu[J];
        uint32_t ww[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * TPC_CA_SWEEP_T;
            uu[j] = -1;
            ww[j] = 0;
            if (k >= n) continue;
            const int32_t h = a + k;
            const int32_t d = dn[h], u = up[h];
            uu[j] = u;
            const bool dprev = d >= pa && d < pb;
            const bool hd = dprev ? pu[d - pa] == (uint32_t)h : (valid_id(d, N) && up[d] == h);
            // a partner up in the row above sets this bit when that row is swept
            const bool hu = (u >= na && u < nb) ? false : (valid_id(u, N) && dn[u] == h);
            uint32_t low = (uint32_t)(h - lo), dist = 0, bot = hd ? 0u : TPC_CA_W_BOT;
            if (hd && dprev && r > r0) {
                const uint32_t w = atomicOr(&pw[d - pa], TPC_CA_W_UP);
                low = w & 0xFFFFFFu;
                dist = ((w >> 24) & 0x1Fu) + 1;
                bot = w & TPC_CA_W_BOT;
            }
            ww[j] = (hd ? TPC_CA_W_DN : 0u) | (hu ? TPC_CA_W_UP : 0u) | bot | (dist << 24) | low;
            ws.claim[h] = ~0ull;
            ws.cc[h] = make_int2(0, -1);
            ws.dlk[h] = hd ? d : -1;
        }
        __syncthreads();
        if (r > r0) {                                 // the row below is complete: its words to pack
            for (int k = tid; k < pb - pa; k += TPC_CA_SWEEP_T) {
                const uint32_t w = pw[k];
                ws.pack[pa + k] = ((unsigned long long)(w >> 30) << 62) | ((w & TPC_CA_W_BOT) ? TPC_CA_BOT : 0ull) |
                                  ((unsigned long long)((w >> 24) & 0x1Fu) << 32) |
                                  (uint32_t)(lo + (int32_t)(w & 0xFFFFFFu));
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int k = tid + j * TPC_CA_SWEEP_T;
            if (k < n) {
                pw[k] = ww[j];
                pu[k] = (uint32_t)uu[j];
            }
        }
        pa = a;
        pb = a + n;
        __syncthreads();
    }
    // up bits of the block's top row from the row above it, then its words
    if (r1 < n_rows) {
        const int a = ro[r1], n = ro[r1 + 1] - a;
        for (int k = tid; k < n; k += TPC_CA_SWEEP_T) {
            const int32_t d = dn[a + k];
            if (d >= pa && d < pb && pu[d - pa] == (uint32_t)(a + k)) atomicOr(&pw[d - pa], TPC_CA_W_UP);
        }
        __syncthreads();
    }
    for (int k = tid; k < pb - pa; k += TPC_CA_SWEEP_T) {
        const uint32_t w = pw[k];
        ws.pack[pa + k] = ((unsigned long long)(w >> 30) << 62) | ((w & TPC_CA_W_BOT) ? TPC_CA_BOT : 0ull) |
                          ((unsigned long long)((w >> 24) & 0x1Fu) << 32) |
                          (uint32_t)(lo + (int32_t)(w & 0xFFFFFFu));
    }
    __syncthreads();                 // LDS reuse by the workgroup's next block
}

// Step 2: the chain tops and the block-local lowest members that are not
// their chain's bottom follow the block-local lowest members down across
// block edges (a lowest member whose kept link leaves the block continues
// below it) to the chain bottom; a lowest member records its bottom and
// position (every member of its block segment adds its distance to it), and
// the top of each chain records the chain length and the cluster above the
// top (the top end candidate) at the bottom and claims the chain's unlinked
// end clusters (chains of >= min_hits - 2
// clusters).  Other members have nothing to do here.
__device__ inline void ca_tops_one(int32_t h, int32_t N, const int32_t *__restrict__ up,
                                   const int32_t *__restrict__ dn, int32_t min_hits, int32_t n_rows,
                                   const CaWs &ws) {
    {
        ws.fbot[h] = -1;                          // set by ca_firsts at a seed's first cluster
        const unsigned long long w0 = ws.pack[h];
        if (!pack_linked(w0)) return;
        const bool top = !(w0 & TPC_CA_UP);
        const bool lowest = pack_node(w0) == h && !(w0 & TPC_CA_BOT);
        if (!top && !lowest) return;
        int32_t bot = pack_node(w0);
        int32_t pos = pack_dist(w0);
        for (int it = 0; it < n_rows && !(w0 & TPC_CA_BOT); ++it) {   // bound: one hop per block
            const int32_t e = valid_id(bot, N) ? ws.dlk[bot] : -1;
            if (e < 0) break;
            const unsigned long long w = ws.pack[e];
            pos += 1 + pack_dist(w);
            bot = pack_node(w);
        }
        if (lowest) ws.mrec[h] = make_int2(bot, pos);
        if (top && valid_id(bot, N)) {                // chain of pos + 1 clusters
            const int32_t m = pos + 1;
            const int32_t et = up[h];
            ws.cc[bot] = make_int2(m, -1);
            ws.cend[bot] = et;
            if (m >= min_hits - 2) {
                const unsigned long long key = claim_key(m, bot);
                const int32_t eb = dn[bot];
                if (valid_id(eb, N) && !pack_linked(ws.pack[eb])) atomicMin(&ws.claim[eb], key);
                if (valid_id(et, N) && !pack_linked(ws.pack[et])) atomicMin(&ws.claim[et], key);
            }
        }
    }
}

__device__ inline void ca_tops_seg(int seg, int32_t N, const int32_t *__restrict__ off,
                                   const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                   int32_t min_hits, int32_t n_rows, const CaWs &ws) {
    const int a = off[seg], b = off[seg + 1];
    if (threadIdx.x == 0) {                       // counted into by ca_firsts
        ws.segcnt[seg] = 0;
        ws.seghits[seg] = 0;
    }
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) ca_tops_one(h, N, up, dn, min_hits, n_rows, ws);
}

// Seed length of the chain with bottom bb (0 if it is no seed).
__device__ inline int32_t seed_len(const int32_t *up, const int32_t *dn, int32_t N, int32_t min_hits,
                                   const CaWs &ws, int32_t bb, int32_t *won_b) {
    int32_t m = ws.cc[bb].x;
    int32_t wb = 0, wt = 0;
    if (m >= min_hits - 2) {
        unsigned long long key = claim_key(m, bb);
        int32_t eb = dn[bb], et = ws.cend[bb];
        wb = (valid_id(eb, N) && ws.claim[eb] == key);
        wt = (valid_id(et, N) && ws.claim[et] == key);
    }
    *won_b = wb;
    int32_t len = m + wb + wt;
    return len >= min_hits ? len : 0;
}

// Seed of the chain with bottom h, recognised there: its first cluster (h,
// or the bottom end below h if h's chain won it) gets the bottom and the
// seed length (fbot, flen; fbot is -1 at every other cluster, from
// ca_tops); returns that first cluster, or -1 if the chain is no seed.  A
// first cluster belongs to one seed at most: a won end has one winner.
__device__ inline int32_t ca_first_one(int32_t h, int32_t N, const int32_t *__restrict__ up,
                                       const int32_t *__restrict__ dn, int32_t min_hits, const CaWs &ws,
                                       int32_t &len) {
    len = 0;
    if (ws.cc[h].x < 2) return -1;               // h is no chain bottom
    int32_t wb;
    const int32_t l = seed_len(up, dn, N, min_hits, ws, h, &wb);
    if (l == 0) return -1;
    const int32_t first = wb ? dn[h] : h;        // a won end is a valid id
    ws.fbot[first] = h;
    ws.flen[first] = l;
    len = l;
    return first;
}

// Rows down from segment seg to the segment of cluster e (a chain bottom's
// bottom end lies one or two rows down in the same frame and sector), 0 for
// e in seg itself; at most TPC_CA_BELOW.
#define TPC_CA_BELOW 2
__device__ inline int rows_below(const int32_t *__restrict__ off, int seg, int32_t e) {
    int d = 0;
    while (d < TPC_CA_BELOW && seg - d > 0 && e < off[seg - d]) ++d;
    return d;
}

// Seeds recognised at the bottoms of segment seg, counted (seeds and hits)
// into the segments of their first clusters: seg itself or up to
// TPC_CA_BELOW rows down (ca_tops zeroed the counts).  Contains barriers:
// call from the whole workgroup.
__device__ inline void ca_firsts_seg(int seg, int32_t N, const int32_t *__restrict__ off,
                                     const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                     int32_t min_hits, const CaWs &ws) {
    __shared__ int acc[2 * (TPC_CA_BELOW + 1)];
    if (threadIdx.x < 2 * (TPC_CA_BELOW + 1)) acc[threadIdx.x] = 0;
    __syncthreads();
    const int a = off[seg], b = off[seg + 1];
    int cnt[TPC_CA_BELOW + 1] = {}, hits[TPC_CA_BELOW + 1] = {};
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) {
        int32_t len;
        const int32_t f = ca_first_one(h, N, up, dn, min_hits, ws, len);
        if (f >= 0) {
            const int d = f == h ? 0 : rows_below(off, seg, f);
#pragma unroll
            for (int q = 0; q <= TPC_CA_BELOW; ++q) {
                cnt[q] += d == q;
                hits[q] += d == q ? len : 0;
            }
        }
    }
#pragma unroll
    for (int q = 0; q <= TPC_CA_BELOW; ++q) {
#pragma unroll
        for (int x = TPC_WAVE / 2; x > 0; x >>= 1) {
            cnt[q] += __shfl_xor(cnt[q], x, TPC_WAVE);
            hits[q] += __shfl_xor(hits[q], x, TPC_WAVE);
        }
    }
    if ((threadIdx.x & (TPC_WAVE - 1)) == 0) {
#pragma unroll
        for (int q = 0; q <= TPC_CA_BELOW; ++q) {
            if (cnt[q]) {
                atomicAdd(&acc[2 * q], cnt[q]);
                atomicAdd(&acc[2 * q + 1], hits[q]);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x <= TPC_CA_BELOW && seg - (int)threadIdx.x >= 0 && acc[2 * threadIdx.x]) {
        atomicAdd(&ws.segcnt[seg - threadIdx.x], acc[2 * threadIdx.x]);
        atomicAdd(&ws.seghits[seg - threadIdx.x], acc[2 * threadIdx.x + 1]);
    }
}

// The same for one wavefront (no barriers; several wavefronts of a
// workgroup may work on different segments).
__device__ inline void ca_firsts_wave(int seg, int32_t N, const int32_t *__restrict__ off,
                                      const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                      int32_t min_hits, const CaWs &ws) {
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int a = off[seg], b = off[seg + 1];
    int cnt[TPC_CA_BELOW + 1] = {}, hits[TPC_CA_BELOW + 1] = {};
    for (int h = a + lane; h < b; h += TPC_WAVE) {
        int32_t len;
        const int32_t f = ca_first_one(h, N, up, dn, min_hits, ws, len);
        if (f >= 0) {
            const int d = f == h ? 0 : rows_below(off, seg, f);
#pragma unroll
            for (int q = 0; q <= TPC_CA_BELOW; ++q) {
                cnt[q] += d == q;
                hits[q] += d == q ? len : 0;
            }
        }
    }
#pragma unroll
    for (int q = 0; q <= TPC_CA_BELOW; ++q) {
#pragma unroll
        for (int x = TPC_WAVE / 2; x > 0; x >>= 1) {
            cnt[q] += __shfl_xor(cnt[q], x, TPC_WAVE);
            hits[q] += __shfl_xor(hits[q], x, TPC_WAVE);
        }
    }
    if (lane <= TPC_CA_BELOW && seg - lane >= 0) {
        int c = 0, hh = 0;
#pragma unroll
        for (int q = 0; q <= TPC_CA_BELOW; ++q) {
            c = lane == q ? cnt[q] : c;
            hh = lane == q ? hits[q] : hh;
        }
        if (c) {
            atomicAdd(&ws.segcnt[seg - lane], c);
            atomicAdd(&ws.seghits[seg - lane], hh);
        }
    }
}

// Record of the seed starting at cluster h (chain bottom fb, length len) as
// seed i with hits from offset o, within capacity.
__device__ inline void ca_place_one(int32_t h, int32_t fb, int32_t len, int i, int o, int32_t N,
                                    const int32_t *__restrict__ up, const float *__restrict__ y,
                                    const float *__restrict__ z, int frame, int sector, int row,
                                    int32_t cap_seeds, int32_t cap_hits, const tpc_seeds &sd, const CaWs &ws,
                                    int32_t *len_hist) {
    if (i < cap_seeds && o + len <= cap_hits) {
        sd.offsets[i] = o;
        sd.offsets[i + 1] = o + len;   // equals the next seed's offset: the placed
                                       // prefix stays well formed on overflow
        sd.frame[i] = frame;
        sd.sector[i] = sector;
        sd.first_row[i] = row;
        const int32_t wb = (h != fb);
        if (wb) {
            sd.hits[o] = h;
            if (sd.hit_yz) put_yz(sd.hit_yz, o, y[h], z[h]);
        }
        const int32_t m = ws.cc[fb].x;
        if (len > m + wb) {
            const int32_t et = ws.cend[fb];
            sd.hits[o + len - 1] = et;
            if (sd.hit_yz && valid_id(et, N)) put_yz(sd.hit_yz, o + len - 1, y[et], z[et]);
        }
        ws.cc[fb].y = o + wb;
        if (len_hist) atomicAdd(&len_hist[len < TPC_MAX_ROWS ? len : TPC_MAX_ROWS], 1);
    }
}

// Contains barriers: call from the whole workgroup.  Returns nothing; seeds
// of the segment go to [segbs[seg], ...) within capacity.
__device__ inline void ca_place_seg(int seg, int32_t N, const int32_t *__restrict__ off,
                                    const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                    const float *__restrict__ y, const float *__restrict__ z,
                                    int32_t n_sectors, int32_t n_rows, int32_t cap_seeds,
                                    int32_t cap_hits, const tpc_seeds &sd, const CaWs &ws,
                                    int32_t *len_hist = nullptr) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    const int a = off[seg], b = off[seg + 1];
    int carry_c = ws.segbs[seg], carry_h = ws.segbh[seg];
    const int frame = seg / (n_sectors * n_rows);
    const int sector = (seg / n_rows) % n_sectors;
    const int row = seg % n_rows;
    for (int base = a; base < b; base += TPC_BLOCK) {
        const int h = base + threadIdx.x;
        int32_t fb = -1, len = 0;
        if (h < b) fb = ws.fbot[h];
        if (fb >= 0) len = ws.flen[h];
        int tc, th;
        int pc = block_exclusive_scan(fb >= 0 ? 1 : 0, sh, &tc);
        int ph = block_exclusive_scan(len, sh, &th);
        if (fb >= 0)
            ca_place_one(h, fb, len, carry_c + pc, carry_h + ph, N, up, y, z, frame, sector, row, cap_seeds,
                         cap_hits, sd, ws, len_hist);
        carry_c += tc;
        carry_h += th;
    }
}

// The same for one wavefront (no barriers; the seeds get the same indices:
// the prefixes run over the segment's clusters in the same order).
__device__ inline void ca_place_wave(int seg, int32_t N, const int32_t *__restrict__ off,
                                     const int32_t *__restrict__ up, const float *__restrict__ y,
                                     const float *__restrict__ z, int32_t n_sectors, int32_t n_rows,
                                     int32_t cap_seeds, int32_t cap_hits, const tpc_seeds &sd, const CaWs &ws,
                                     int32_t *len_hist) {
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int a = off[seg], b = off[seg + 1];
    int carry_c = ws.segbs[seg], carry_h = ws.segbh[seg];
    const int frame = seg / (n_sectors * n_rows);
    const int sector = (seg / n_rows) % n_sectors;
    const int row = seg % n_rows;
    for (int base = a; base < b; base += TPC_WAVE) {
        const int h = base + lane;
        int32_t fb = -1, len = 0;
        if (h < b) fb = ws.fbot[h];
        if (fb >= 0) len = ws.flen[h];
        const int f = fb >= 0 ? 1 : 0;
        const int ic = wave_inclusive_scan(f), ih = wave_inclusive_scan(len);
        if (fb >= 0)
            ca_place_one(h, fb, len, carry_c + ic - f, carry_h + ih - len, N, up, y, z, frame, sector, row,
                         cap_seeds, cap_hits, sd, ws, len_hist);
        carry_c += __shfl(ic, TPC_WAVE - 1, TPC_WAVE);
        carry_h += __shfl(ih, TPC_WAVE - 1, TPC_WAVE);
    }
}

// Every chain member writes itself into its seed: its chain's bottom and
// its position from it come from its block-local lowest member (the bottom
// itself, or the record ca_tops left there) and its distance to that member.
__device__ inline void ca_members_one(int32_t h, int32_t N, const float *__restrict__ y,
                                      const float *__restrict__ z, int32_t cap_hits, const tpc_seeds &sd,
                                      const CaWs &ws) {
    {
        const unsigned long long w = ws.pack[h];
        if (!pack_linked(w)) return;
        int32_t bb = pack_node(w), k = pack_dist(w);
        if (!(w & TPC_CA_BOT)) {
            if (!valid_id(bb, N)) return;
            const int2 r = ws.mrec[bb];
            bb = r.x;
            k += r.y;
        }
        if (!valid_id(bb, N)) return;
        const int2 c = ws.cc[bb];                    // (chain length, core offset)
        const int32_t o = c.y;
        if (o >= 0 && k >= 0 && k < c.x && o + k < cap_hits) {
            sd.hits[o + k] = h;
            if (sd.hit_yz) put_yz(sd.hit_yz, o + k, y[h], z[h]);
        }
    }
}

__device__ inline void ca_members_seg(int seg, int32_t N, const int32_t *__restrict__ off,
                                      const int32_t *__restrict__ up, const int32_t *__restrict__ dn,
                                      const float *__restrict__ y, const float *__restrict__ z,
                                      int32_t cap_hits, const tpc_seeds &sd, const CaWs &ws) {
    const int a = off[seg], b = off[seg + 1];
    for (int h = a + threadIdx.x; h < b; h += TPC_BLOCK) ca_members_one(h, N, y, z, cap_hits, sd, ws);
}

}  // namespace tpc_ca
