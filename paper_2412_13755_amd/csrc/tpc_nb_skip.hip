// Neighbours across a missing pad row (gfx950).  After the adjacent-row
// search, each cluster it left without partners looks for them up to two
// rows away: the best pair spanning three rows ((A, B) = (1, 2) or (2, 1)
// rows below/above), else the best spanning four ((2, 2)); the exact
// predicates and the ordering are those of best_pair.  A cluster that has
// an adjacent-row triplet keeps it, so only the unlinked ones are queried.
//
//  skip_bin    global cell-sorted copy of every row lying within two rows
//              of an h-row whose four partner rows do not all fit the LDS
//              form (rare: rows of more than SKIP_LDS_ROW clusters)
//  skip_query  one workgroup per h-row: returns at once when all its
//              clusters are linked; otherwise rows r-1/r+1 and r-2/r+2 are
//              binned as two LDS row pairs (one coalesced read each), the
//              unlinked clusters are compacted so that consecutive lanes
//              query, and each query reads only LDS.
#include "tpc_nb_device.hpp"
#include "tpc_nb_skip.hpp"

namespace {

#define SKIP_LDS_ROW 512
#define SKIP_LDS_CELLS 1024
using SkipPair = tpc_nb::PairLdsT<SKIP_LDS_ROW, SKIP_LDS_CELLS>;

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

// Does interior h-row seg read its partner rows from the global copies?
__device__ inline bool skip_global(const int32_t *off, int seg, int n_rows) {
    const int r = seg % n_rows;
    if (r < 1 || r > n_rows - 2) return false;
    int m = 0;
    for (int dr = -2; dr <= 2; ++dr) {
        if (dr == 0) continue;
        int a, b;
        partner_row(off, seg, r, n_rows, dr, a, b);
        m = b - a > m ? b - a : m;
    }
    return m > SKIP_LDS_ROW;
}

__global__ void __launch_bounds__(TPC_BLOCK)
skip_bin(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
         const float *__restrict__ z, float win_y, float win_z, SegGrid *grid, int32_t *cstart, float *sy,
         float *sz, int32_t *sid) {
    __shared__ tpc_nb::BinLds L;
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    const int r = seg % n_rows;
    bool need = false;
    for (int k = -2; k <= 2; ++k) {
        const int rh = r + k;                       // an h-row k rows from this one
        if (k != 0 && rh >= 1 && rh <= n_rows - 2) need = need || skip_global(off, seg + k, n_rows);
    }
    if (!need) return;
    const int a = off[seg], b = off[seg + 1], n = b - a;
    const int base = a + seg;
    if (n == 0) {
        if (threadIdx.x == 0) {
            grid[seg] = SegGrid{0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
            cstart[base] = a;
        }
        return;
    }
    float ext[4];
    tpc_nb::row_extent(y, z, a, b, L.red, ext);
    const SegGrid g = tpc_nb::row_grid(ext[0], ext[1], ext[2], ext[3], n, TPC_CELL_CAP, win_y, win_z);
    if (threadIdx.x == 0) grid[seg] = g;
    tpc_nb::row_sort(y, z, a, b, g, L.cnt, L.scan_sh, sy, sz, sid, cstart + base, a);
}

// Best pair across one missing row for cluster (hy, hz): (1, 2) and (2, 1)
// compete by (q, u, d); (2, 2) only if neither passes.  R1/R2 hold the row
// pairs r-1/r+1 and r-2/r+2 as (down, up) views.
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

// A cell-sorted row as best_pair reads it.
template <class FP, class IP>
struct RowView {
    FP y, z;
    IP i;
    const int32_t *cs;
    SegGrid g;
    int32_t base;
};

__global__ void __launch_bounds__(TPC_BLOCK)
skip_query(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
           const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z,
           const SegGrid *grid, const int32_t *cstart, const float *sy, const float *sz, const int32_t *sid,
           int32_t *up, int32_t *dn) {
    __shared__ SkipPair L1, L2;
    __shared__ int32_t qlist[TPC_BLOCK];
    __shared__ int qsh[TPC_BLOCK / TPC_WAVE];
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    const int r = seg % n_rows;
    if (r < 1 || r > n_rows - 2) return;
    const bool lo2 = r >= 2, hi2 = r <= n_rows - 3;
    if (!lo2 && !hi2) return;
    const int a = off[seg], b = off[seg + 1];
    if (a == b) return;
    int any = 0;
    for (int i = a + (int)threadIdx.x; i < b; i += TPC_BLOCK) any |= up[i] < 0;
    if (!__syncthreads_or(any)) return;
    int ra[4], rb[4];                     // rows r-2, r-1, r+1, r+2
    partner_row(off, seg, r, n_rows, -2, ra[0], rb[0]);
    partner_row(off, seg, r, n_rows, -1, ra[1], rb[1]);
    partner_row(off, seg, r, n_rows, 1, ra[2], rb[2]);
    partner_row(off, seg, r, n_rows, 2, ra[3], rb[3]);
    const bool global = skip_global(off, seg, n_rows);
    using LV = RowView<const float *, const uint16_t *>;
    using GV = RowView<const float *, const int32_t *>;
    LV l[4];
    GV gv[4];
    if (!global) {
        SegGrid gd1, gu1, gd2, gu2;
        int C1, C2;
        tpc_nb::pair_bin(y, z, ra[1], rb[1], ra[2], rb[2], win_y, win_z, L1, gd1, gu1, C1);
        tpc_nb::pair_bin(y, z, ra[0], rb[0], ra[3], rb[3], win_y, win_z, L2, gd2, gu2, C2);
        l[0] = LV{L2.y, L2.z, L2.rel, L2.cs, gd2, ra[0]};
        l[1] = LV{L1.y, L1.z, L1.rel, L1.cs, gd1, ra[1]};
        l[2] = LV{L1.y, L1.z, L1.rel, L1.cs + C1, gu1, ra[2]};
        l[3] = LV{L2.y, L2.z, L2.rel, L2.cs + C2, gu2, ra[3]};
    } else {
        const SegGrid none = {0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
        const int dr[4] = {-2, -1, 1, 2};
        for (int k = 0; k < 4; ++k) {
            const bool ex = (k == 0 && lo2) || k == 1 || k == 2 || (k == 3 && hi2);
            const int s = seg + dr[k];
            gv[k] = GV{sy, sz, sid, ex ? cstart + off[s] + s : cstart, ex ? grid[s] : none, 0};
        }
    }
    for (int base = a; base < b; base += TPC_BLOCK) {
        const int h = base + (int)threadIdx.x;
        const int unl = h < b && up[h] < 0;
        int cnt;
        const int pos = block_exclusive_scan(unl, qsh, &cnt);
        if (unl) qlist[pos] = h;
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int32_t q = qlist[threadIdx.x];
            const float hy = y[q], hz = z[q];
            const tpc_nb::Best bt = global
                ? skip_pair(hy, hz, gv[1], gv[2], gv[0], gv[3], lo2, hi2, win_y, win_z, cut_y, cut_z)
                : skip_pair(hy, hz, l[1], l[2], l[0], l[3], lo2, hi2, win_y, win_z, cut_y, cut_z);
            if (bt.u >= 0) {
                up[q] = bt.u;
                dn[q] = bt.d;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_neighbours_skip(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                                  const NbWs &ws, hipStream_t st) {
    hipError_t e = launch_neighbours(ctx, fr, up, dn, ws, st);
    if (e != hipSuccess) return e;
    const int NR = fr->n_frames * ctx->cfg.n_sectors * ctx->cfg.n_rows;
    const tpc_config &c = ctx->cfg;
    hipLaunchKernelGGL(skip_bin, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y, fr->z,
                       c.win_y, c.win_z, ws.grid, ws.cstart, ws.sy, ws.sz, ws.sid);
    hipLaunchKernelGGL(skip_query, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y, fr->z,
                       c.win_y, c.win_z, c.cut_y, c.cut_z, ws.grid, ws.cstart, ws.sy, ws.sz, ws.sid, up, dn);
    return hipGetLastError();
}
