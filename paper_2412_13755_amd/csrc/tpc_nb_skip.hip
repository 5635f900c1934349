// Neighbours across a missing pad row (gfx950).  After the adjacent-row
// search, each cluster it left without partners looks for them up to two
// rows away: the best pair spanning three rows ((A, B) = (1, 2) or (2, 1)
// rows below/above), else the best spanning four ((2, 2)); the exact
// predicates and the ordering are those of best_pair.  A cluster that has
// an adjacent-row triplet keeps it, so only the unlinked ones are queried --
// a tenth to a quarter of the clusters, spread over every row (noise, track
// ends, the clusters beside a missing one), thirty to sixty per row.
//
//  skip_seg    one workgroup per h-row whose partner rows hold at most
//              SKIP_ROW_MAX clusters each, taking the row's clusters in
//              chunks of SKIP_Q; rows in ascending order over all sectors,
//              so that the inner rows, which hold the most clusters, do not
//              trail.  A chunk's unlinked clusters with finite coordinates
//              (the others cannot link) go to LDS, ranked by y; every thread
//              streams clusters of the four partner rows (coalesced) and
//              finds the queries in its window by a binary search over the
//              ranked y -- exact, since rounding is monotonic, so the y
//              predicate |fl(y_h - y_c)| <= w holds on a contiguous run of
//              ranks -- once to count each query's candidates per row, once
//              more to store them (row position and coordinates) in
//              exact-size lists carved from an LDS pool by a prefix sum;
//              then a thread per query scores the (down, up) pairs of its
//              lists, from LDS only, with the exact arithmetic of best_pair.
//              A chunk whose lists exceed the pool (far beyond any TPC
//              occupancy) scans the two rows per query instead.
//  skip_zero, skip_prep, skip_query
//              the h-rows with a larger partner row: global cell-sorted
//              copies of the rows they need, their unlinked clusters in one
//              list, one thread per listed cluster running best_pair in the
//              sorted copies.
#include "tpc_nb_device.hpp"
#include "tpc_nb_skip.hpp"

namespace {

// Best pair across one missing row for cluster (hy, hz): (1, 2) and (2, 1)
// compete by (q, u, d); (2, 2) only if neither passes.  d1, u1, d2, u2 are
// the rows r-1, r+1, r-2, r+2 (d2 only if lo2, u2 only if hi2).
template <class V>
__device__ inline tpc_nb::Best skip_pair(float hy, float hz, const V &d1, const V &u1, const V &d2,
                                         const V &u2, bool lo2, bool hi2, float win_y, float win_z,
                                         float cut_y, float cut_z) {
    tpc_nb::Best bt = {0.f, -1, -1};
    if (hi2)
        bt = tpc_nb::best_pair<1, 2>(hy, hz, u2.y, u2.z, u2.i, u2.cs, u2.g, u2.base, d1.y, d1.z, d1.i, d1.cs,
                                     d1.g, d1.base, win_y, win_z, cut_y, cut_z);
    if (lo2) {
        const tpc_nb::Best c = tpc_nb::best_pair<2, 1>(hy, hz, u1.y, u1.z, u1.i, u1.cs, u1.g, u1.base, d2.y,
                                                       d2.z, d2.i, d2.cs, d2.g, d2.base, win_y, win_z,
                                                       cut_y, cut_z);
        if (c.u >= 0 && tpc_nb::better(c.q, c.u, c.d, bt)) bt = c;
    }
    if (bt.u < 0 && lo2 && hi2)
        bt = tpc_nb::best_pair<2, 2>(hy, hz, u2.y, u2.z, u2.i, u2.cs, u2.g, u2.base, d2.y, d2.z, d2.i, d2.cs,
                                     d2.g, d2.base, win_y, win_z, cut_y, cut_z);
    return bt;
}

// A cell-sorted row as best_pair reads it (global copy: stored ids are
// global cluster ids, base 0).
struct RowView {
    const float *y, *z;
    const int32_t *i;
    const int32_t *cs;
    SegGrid g;
    int32_t base;
};

__device__ inline RowView row_view(const SkipWs &w, const int32_t *off, int s) {
    return RowView{w.nb.sy, w.nb.sz, w.nb.sid, w.nb.cstart + off[s] + s, w.nb.grid[s], 0};
}

#define SKIP_ROW_MAX 1024      // partner rows up to this size: skip_seg
#define SKIP_Q 128             // queries per skip_seg pass
#define SKIP_POOL 1024         // window candidates of one pass, all queries and rows

// Cluster range of row r + dr of h-row seg's (frame, sector); empty if that
// row is outside the sector.
__device__ inline void partner_row(const int32_t *off, int seg, int r, int n_rows, int dr, int &a, int &b) {
    const int rr = r + dr;
    if (rr < 0 || rr >= n_rows) {
        a = b = 0;
        return;
    }
    a = off[seg + dr];
    b = off[seg + dr + 1];
}

// Does interior h-row seg have a partner row too large for skip_seg?
__device__ inline bool skip_large(const int32_t *off, int seg, int n_rows) {
    const int r = seg % n_rows;
    if (r < 1 || r > n_rows - 2) return false;
    int m = 0;
    for (int dr = -2; dr <= 2; ++dr) {
        if (dr == 0) continue;
        int a, b;
        partner_row(off, seg, r, n_rows, dr, a, b);
        m = b - a > m ? b - a : m;
    }
    return m > SKIP_ROW_MAX;
}

__global__ void skip_zero(int32_t *count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0;
}

// Cell-sorted copy of every row that a large h-row needs; the unlinked
// clusters of large h-rows appended to the list.
__global__ void __launch_bounds__(TPC_BLOCK)
skip_prep(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
          const float *__restrict__ z, float win_y, float win_z, const int32_t *__restrict__ up, SkipWs w) {
    __shared__ tpc_nb::BinLds L;
    __shared__ int base_sh;
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    const int r = seg % n_rows;
    bool need = false;
    for (int k = -2; k <= 2; ++k) {
        const int rh = r + k;                       // an h-row k rows from this one
        if (k != 0 && rh >= 1 && rh <= n_rows - 2) need = need || skip_large(off, seg + k, n_rows);
    }
    const int a = off[seg], b = off[seg + 1], n = b - a;
    if (need) {
        const int cbase = a + seg;
        if (n == 0) {
            if (threadIdx.x == 0) {
                w.nb.grid[seg] = SegGrid{0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
                w.nb.cstart[cbase] = a;
            }
        } else {
            float ext[4];
            tpc_nb::row_extent(y, z, a, b, L.red, ext);
            const SegGrid g = tpc_nb::row_grid(ext[0], ext[1], ext[2], ext[3], n, TPC_CELL_CAP, win_y, win_z);
            if (threadIdx.x == 0) w.nb.grid[seg] = g;
            tpc_nb::row_sort(y, z, a, b, g, L.cnt, L.scan_sh, w.nb.sy, w.nb.sz, w.nb.sid, w.nb.cstart + cbase, a);
        }
    }
    if (!skip_large(off, seg, n_rows) || (r < 2 && r > n_rows - 3)) return;
    for (int c0 = a; c0 < b; c0 += TPC_BLOCK) {
        const int h = c0 + (int)threadIdx.x;
        const int unl = h < b && up[h] < 0;
        int cnt;
        const int pos = block_exclusive_scan(unl, L.scan_sh, &cnt);
        if (threadIdx.x == 0 && cnt > 0) base_sh = atomicAdd(w.count, cnt);
        __syncthreads();
        if (unl) w.list[base_sh + pos] = make_int2(h, seg);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
skip_query(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
           const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z, SkipWs w,
           int32_t *up, int32_t *dn) {
    const int count = *w.count;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < count; i += gridDim.x * TPC_BLOCK) {
        const int2 e = w.list[i];
        const int32_t h = e.x;
        const int seg = e.y;
        const int r = seg % n_rows;
        const bool lo2 = r >= 2, hi2 = r <= n_rows - 3;
        const RowView d1 = row_view(w, off, seg - 1), u1 = row_view(w, off, seg + 1);
        const RowView d2 = lo2 ? row_view(w, off, seg - 2) : d1;
        const RowView u2 = hi2 ? row_view(w, off, seg + 2) : u1;
        const tpc_nb::Best bt = skip_pair(y[h], z[h], d1, u1, d2, u2, lo2, hi2, win_y, win_z, cut_y, cut_z);
        if (bt.u >= 0) {
            up[h] = bt.u;
            dn[h] = bt.d;
        }
    }
}

// Scores pair (d, u) for h exactly as best_pair does (the windows already
// passed) and keeps the better one.
template <int A, int B>
__device__ inline void score_pair(float hy, float hz, float yu, float zu, int32_t u, float yd, float zd,
                                  int32_t d, float cut_y, float cut_z, tpc_nb::Best &best) {
#pragma clang fp contract(off)
    constexpr float fa = (float)A, fb = (float)B;
    constexpr float g = 2.0f / (float)(A + B);
    const float ay = yu - hy, az = zu - hz;
    const float by = hy - yd, bz = hz - zd;
    const float ty = ay / fb, tz = az / fb;
    const float sy = by / fa, sz = bz / fa;
    const float ey = ty - sy;
    const float ez = tz - sz;
    const float dy = g * ey;
    const float dz = g * ez;
    if (!(fabsf(dy) <= cut_y && fabsf(dz) <= cut_z)) return;
    const float qy = dy * dy;
    const float qz = dz * dz;
    const float q = qy + qz;
    if (tpc_nb::better(q, u, d, best)) { best.q = q; best.u = u; best.d = d; }
}

// Every pair of the down row [d0, d1) (A rows below) and up row [u0, u1)
// (B rows above) inside the windows: the exact scan for an overflowing list.
template <int A, int B>
__device__ inline void scan_rows(float hy, float hz, const float *__restrict__ y, const float *__restrict__ z,
                                 int d0, int d1, int u0, int u1, float win_y, float win_z, float cut_y,
                                 float cut_z, tpc_nb::Best &best) {
#pragma clang fp contract(off)
    constexpr float fa = (float)A, fb = (float)B;
    for (int u = u0; u < u1; ++u) {
        const float yu = y[u], zu = z[u];
        const float ay = yu - hy, az = zu - hz;
        if (!(fabsf(ay) <= fb * win_y && fabsf(az) <= fb * win_z)) continue;
        for (int d = d0; d < d1; ++d) {
            const float yd = y[d], zd = z[d];
            const float by = hy - yd, bz = hz - zd;
            if (!(fabsf(by) <= fa * win_y && fabsf(bz) <= fa * win_z)) continue;
            score_pair<A, B>(hy, hz, yu, zu, u, yd, zd, d, cut_y, cut_z, best);
        }
    }
}

struct SegLds {
    float qy[SKIP_Q], qz[SKIP_Q];
    int32_t qh[SKIP_Q];
    float ry[SKIP_Q];                    // query y in ascending order
    int32_t rq[SKIP_Q];                  // ... and the query at each rank
    int32_t cnt[4 * SKIP_Q];             // candidates of (row k, query q) at k * SKIP_Q + q
    uint16_t start[4 * SKIP_Q];          // their list's start in the pool
    float py[SKIP_POOL], pz[SKIP_POOL];  // candidate coordinates
    uint16_t pool[SKIP_POOL];            // candidate positions within the partner row
    int scan_sh[TPC_BLOCK / TPC_WAVE];
};

// Best pair of query q from its lists of down row kd (A below) and up row ku
// (B above); ra: first cluster of each partner row.
template <int A, int B>
__device__ inline void pairs_of(const SegLds &L, int q, int kd, int ku, const int ra[4], const int rb[4],
                                bool listed, float hy, float hz, const float *__restrict__ y,
                                const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z,
                                tpc_nb::Best &best) {
    if (!listed) {
        scan_rows<A, B>(hy, hz, y, z, ra[kd], rb[kd], ra[ku], rb[ku], win_y, win_z, cut_y, cut_z, best);
        return;
    }
    const int d0 = L.start[kd * SKIP_Q + q], nd = L.cnt[kd * SKIP_Q + q];
    const int u0 = L.start[ku * SKIP_Q + q], nu = L.cnt[ku * SKIP_Q + q];
    for (int iu = 0; iu < nu; ++iu) {
        const int32_t u = ra[ku] + L.pool[u0 + iu];
        const float yu = L.py[u0 + iu], zu = L.pz[u0 + iu];
        for (int id = 0; id < nd; ++id) {
            const int32_t d = ra[kd] + L.pool[d0 + id];
            score_pair<A, B>(hy, hz, yu, zu, u, L.py[d0 + id], L.pz[d0 + id], d, cut_y, cut_z, best);
        }
    }
}

// The queries whose window holds partner-row cluster (cy, cz): counted
// (FILL = false) or stored at the cursors cnt (FILL = true).  Queries are
// ranked by y; fl(hy - cy) does not decrease with hy, so the ones passing
// |fl(hy - cy)| <= wy are a run of ranks, found by a binary search for its
// first member.  The predicates are those of best_pair: hy - cy for a row
// below (by = y_h - y_d), cy - hy for a row above (ay = y_u - y_h), whose
// magnitudes are equal.
template <bool FILL>
__device__ inline void window_hits(SegLds &L, int nq, int k, int rel, float cy, float cz, float wy, float wz) {
#pragma clang fp contract(off)
    int lo = 0, hi = nq;                     // first rank with hy - cy >= -wy
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L.ry[mid] - cy >= -wy) hi = mid;
        else lo = mid + 1;
    }
    for (int j = lo; j < nq; ++j) {
        const float hy = L.ry[j];
        const float dy = k < 2 ? hy - cy : cy - hy;
        if (!(fabsf(dy) <= wy)) break;
        const int q = L.rq[j];
        const float hz = L.qz[q];
        const float dz = k < 2 ? hz - cz : cz - hz;
        if (fabsf(dz) <= wz) {
            const int slot = atomicAdd(&L.cnt[k * SKIP_Q + q], 1);
            if (FILL) {
                L.pool[slot] = (uint16_t)rel;
                L.py[slot] = cy;
                L.pz[slot] = cz;
            }
        }
    }
}

template <bool FILL>
__device__ inline void window_pass(SegLds &L, int nq, const int ra[4], const int rb[4],
                                   const float *__restrict__ y, const float *__restrict__ z, float win_y,
                                   float win_z) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float sc = (k == 0 || k == 3) ? 2.0f : 1.0f;     // rows away
        const float wy = sc * win_y, wz = sc * win_z;
        for (int c = ra[k] + (int)threadIdx.x; c < rb[k]; c += TPC_BLOCK) {
            const float cy = y[c], cz = z[c];
            if (isfinite(cy)) window_hits<FILL>(L, nq, k, c - ra[k], cy, cz, wy, wz);
        }
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
skip_seg(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
         const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z, int32_t *up,
         int32_t *dn) {
#pragma clang fp contract(off)
    __shared__ SegLds L;
    // rows in ascending order over all sectors: the inner rows, which hold
    // the most clusters (loopers) and take longest, start first; blocks go
    // round-robin over the XCDs, so each gets a share of every row
    const int n_fs = gridDim.x / n_rows;
    const int r = blockIdx.x / n_fs;
    const int seg = (blockIdx.x % n_fs) * n_rows + r;
    if (r < 1 || r > n_rows - 2) return;
    const bool lo2 = r >= 2, hi2 = r <= n_rows - 3;
    if (!lo2 && !hi2) return;
    const int a = off[seg], b = off[seg + 1];
    if (a == b || skip_large(off, seg, n_rows)) return;
    int ra[4], rb[4];                         // rows r-2, r-1, r+1, r+2
    partner_row(off, seg, r, n_rows, -2, ra[0], rb[0]);
    partner_row(off, seg, r, n_rows, -1, ra[1], rb[1]);
    partner_row(off, seg, r, n_rows, 1, ra[2], rb[2]);
    partner_row(off, seg, r, n_rows, 2, ra[3], rb[3]);
    const int tid = threadIdx.x;
    constexpr int PER = 4 * SKIP_Q / TPC_BLOCK;         // list counts per thread in the scan
    for (int c0 = a; c0 < b; c0 += SKIP_Q) {
        const int h = c0 + tid;
        int uh = 0;
        float hy0 = 0.f, hz0 = 0.f;
        if (tid < SKIP_Q && h < b) {
            uh = up[h];
            hy0 = y[h];
            hz0 = z[h];
        }
        // unlinked and finite (a non-finite cluster never links)
        const int unl = tid < SKIP_Q && h < b && uh < 0 && isfinite(hy0) && isfinite(hz0);
        int nq;
        const int pos = block_exclusive_scan(unl, L.scan_sh, &nq);
        if (nq == 0) continue;                // uniform
        if (unl) {
            L.qh[pos] = h;
            L.qy[pos] = hy0;
            L.qz[pos] = hz0;
        }
        for (int k = tid; k < 4 * SKIP_Q; k += TPC_BLOCK) L.cnt[k] = 0;
        __syncthreads();
        // rank by y (ties by position): a permutation, as every y is finite
        if (tid < nq) {
            const float v = L.qy[tid];
            int rk = 0;
            for (int j = 0; j < nq; ++j) {
                const float w = L.qy[j];
                rk += (w < v) | ((w == v) & (j < tid));
            }
            L.ry[rk] = v;
            L.rq[rk] = tid;
        }
        __syncthreads();
        window_pass<false>(L, nq, ra, rb, y, z, win_y, win_z);
        __syncthreads();
        // list starts: exclusive prefix of the counts (thread t owns PER of them)
        int v[PER], local = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            v[j] = L.cnt[tid * PER + j];
            local += v[j];
        }
        int total;
        int run = block_exclusive_scan(local, L.scan_sh, &total);
        const bool listed = total <= SKIP_POOL;   // uniform
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            L.start[tid * PER + j] = (uint16_t)(listed ? run : 0);
            L.cnt[tid * PER + j] = run;           // cursor of the fill pass
            run += v[j];
        }
        __syncthreads();
        if (listed) {
            window_pass<true>(L, nq, ra, rb, y, z, win_y, win_z);
            __syncthreads();
            // cursors have moved to the ends: back to counts
#pragma unroll
            for (int j = 0; j < PER; ++j) L.cnt[tid * PER + j] -= L.start[tid * PER + j];
            __syncthreads();
        }
        if (tid < nq) {
            const float hy = L.qy[tid], hz = L.qz[tid];
            tpc_nb::Best bt = {0.f, -1, -1};
            if (hi2) pairs_of<1, 2>(L, tid, 1, 3, ra, rb, listed, hy, hz, y, z, win_y, win_z, cut_y, cut_z, bt);
            if (lo2) {
                tpc_nb::Best c = {0.f, -1, -1};
                pairs_of<2, 1>(L, tid, 0, 2, ra, rb, listed, hy, hz, y, z, win_y, win_z, cut_y, cut_z, c);
                if (c.u >= 0 && tpc_nb::better(c.q, c.u, c.d, bt)) bt = c;
            }
            if (bt.u < 0 && lo2 && hi2)
                pairs_of<2, 2>(L, tid, 0, 3, ra, rb, listed, hy, hz, y, z, win_y, win_z, cut_y, cut_z, bt);
            if (bt.u >= 0) {
                const int32_t hq = L.qh[tid];
                up[hq] = bt.u;
                dn[hq] = bt.d;
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t skip_ws_layout(void *ws, int64_t N, int64_t NR, SkipWs *out) {
    const size_t nb = nb_ws_layout(ws, N, NR, out ? &out->nb : nullptr);
    WsCarver w(ws ? (void *)((char *)ws + nb) : nullptr);
    int2 *list = w.take<int2>(N > 0 ? N : 1);
    int32_t *count = w.take<int32_t>(1);
    if (out) {
        out->list = list;
        out->count = count;
    }
    return nb + ((w.off + 255) & ~size_t(255));
}

hipError_t launch_neighbours_skip(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                                  const SkipWs &ws, hipStream_t st) {
    hipError_t e = launch_neighbours(ctx, fr, up, dn, ws.nb, st);
    if (e != hipSuccess) return e;
    const int NR = fr->n_frames * ctx->cfg.n_sectors * ctx->cfg.n_rows;
    const tpc_config &c = ctx->cfg;
    hipLaunchKernelGGL(skip_seg, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y, fr->z,
                       c.win_y, c.win_z, c.cut_y, c.cut_z, up, dn);
    hipLaunchKernelGGL(skip_zero, dim3(1), dim3(64), 0, st, ws.count);
    hipLaunchKernelGGL(skip_prep, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y, fr->z,
                       c.win_y, c.win_z, up, ws);
    int blocks = (int)(fr->n_clusters / (8 * TPC_BLOCK)) + 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(skip_query, dim3(blocks), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y,
                       fr->z, c.win_y, c.win_z, c.cut_y, c.cut_z, ws, up, dn);
    return hipGetLastError();
}
