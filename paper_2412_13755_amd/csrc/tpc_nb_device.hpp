#pragma once
// Neighbour finding between adjacent pad rows (gfx950): per-segment device
// functions, used by the stage kernels and by the persistent kernel.
//
// Exact definition (the result every enumeration must reproduce): for each
// cluster h of row r in [1, R-2], the pair (d in row r-1, u in row r+1) that
// passes the position windows and the second-difference cuts with the
// smallest q = dy*dy + dz*dz, ties to the smaller u id, then the smaller d id.
// Every floating-point operation is one single-precision rounding: the
// functions below carry "fp contract(off)" and the stage file is compiled
// with -ffp-contract=off, so no multiply-add is fused.
//
// Design: one workgroup per h-row (frame, sector, row) segment.  Each of
// the two neighbouring rows is put on a y-z cell grid sized from the data
// and counting-sorted by cell; then every thread takes clusters h of its row
// and scans the up-row cells that overlap its window, and for each up
// candidate in the window, the down-row cells that overlap the cut interval
// around the straight-line prediction.  Rows of up to TPC_LDS_ROW clusters
// are binned by the query workgroup itself into LDS, both rows in one
// counting sort with up to four cells per cluster (the row pair is read
// once, coalesced, and every candidate access is an LDS access).
//
// Dense rows (a neighbouring row of more than TPC_LDS_ROW clusters, as in a
// continuous-readout time frame with ~10^4 clusters per pad row): the h-row
// and both neighbouring rows are first counting-sorted by z alone into a
// global copy (nb_bin_seg).  The query workgroup then walks its h-row in
// slabs of consecutive sorted clusters (nearby z); a slab's window in z
// selects a contiguous range of each neighbouring row's sorted copy, which
// is binned into LDS exactly as a small row pair, and the slab's clusters
// are searched there.  A slab whose ranges exceed the LDS is halved; a
// slab of the smallest size that still does not fit is searched directly
// in the global sorted copies.  The cells scanned are derived from the
// window and cut intervals with a safety margin (see best_pair), so they
// over-cover the candidates and the exact predicates decide.
#include "tpc_internal.hpp"

namespace tpc_nb {


// Cell index of coordinate v on an axis of n cells starting at v0, 1/edge iw
// (iw = 0 when n = 1).  Monotonic non-decreasing in v; NaN and values below
// the axis go to cell 0, values beyond it (+inf too) to cell n - 1.
// Branch-free: fmaxf returns the number when the other operand is NaN.
__device__ inline int cell_coord(float v, float v0, float iw, int n) {
#pragma clang fp contract(off)
    float c = (v - v0) * iw;
    c = fmaxf(c, 0.0f);
    c = fminf(c, (float)(n - 1));
    return (int)c;                                  // floor for c >= 0
}

// Grid of one row: cell edges >= edge x the window (1.01 by default), at
// most min(n, cap) cells.  ext = (ymin, ymax, zmin, zmax) of the finite
// coordinates.
__device__ inline SegGrid row_grid(float ymin, float ymax, float zmin, float zmax, int n, int cap,
                                   float win_y, float win_z, float edge = 1.01f) {
#pragma clang fp contract(off)
    if (!(ymin <= ymax)) { ymin = 0.f; ymax = 0.f; }
    if (!(zmin <= zmax)) { zmin = 0.f; zmax = 0.f; }
    const int c = n < cap ? n : cap;
    const float ry = ymax - ymin, rz = zmax - zmin;
    const float fz = rz / (edge * win_z), fy = ry / (edge * win_y);
    const int nzmax = fz >= (float)c ? c : (fz >= 1.0f ? (int)fz : 1);
    const int nymax = fy >= (float)c ? c : (fy >= 1.0f ? (int)fy : 1);
    const int nz = nzmax;
    int ny = c / nz;
    if (ny > nymax) ny = nymax;
    if (ny < 1) ny = 1;
    SegGrid g = {ymin, zmin, ny > 1 ? (float)ny / ry : 0.f, nz > 1 ? (float)nz / rz : 0.f, ny, nz, 0, 0};
    return g;
}

// Finite extent of clusters [a, b) (whole workgroup; contains barriers).
__device__ inline void row_extent(const float *__restrict__ y, const float *__restrict__ z, int a, int b,
                                  float (*red)[TPC_BLOCK / TPC_WAVE], float ext[4]) {
    float ymin = INFINITY, ymax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    for (int i = a + (int)threadIdx.x; i < b; i += TPC_BLOCK) {
        const float yv = y[i], zv = z[i];
        if (isfinite(yv)) { ymin = fminf(ymin, yv); ymax = fmaxf(ymax, yv); }
        if (isfinite(zv)) { zmin = fminf(zmin, zv); zmax = fmaxf(zmax, zv); }
    }
    ymin = wave_min(ymin); ymax = wave_max(ymax);
    zmin = wave_min(zmin); zmax = wave_max(zmax);
    const int wid = threadIdx.x / TPC_WAVE, lane = threadIdx.x & (TPC_WAVE - 1);
    __syncthreads();
    if (lane == 0) { red[0][wid] = ymin; red[1][wid] = ymax; red[2][wid] = zmin; red[3][wid] = zmax; }
    __syncthreads();
    ymin = red[0][0]; ymax = red[1][0]; zmin = red[2][0]; zmax = red[3][0];
    for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w) {
        ymin = fminf(ymin, red[0][w]); ymax = fmaxf(ymax, red[1][w]);
        zmin = fminf(zmin, red[2][w]); zmax = fmaxf(zmax, red[3][w]);
    }
    ext[0] = ymin; ext[1] = ymax; ext[2] = zmin; ext[3] = zmax;
}

// Finite z extent of clusters [a, b) (whole workgroup; contains barriers).
__device__ inline void row_zextent(const float *__restrict__ z, int a, int b, float (*red)[TPC_BLOCK / TPC_WAVE],
                                   float &zlo, float &zhi) {
    float zmin = INFINITY, zmax = -INFINITY;
    for (int i = a + (int)threadIdx.x; i < b; i += TPC_BLOCK) {
        const float zv = z[i];
        if (isfinite(zv)) { zmin = fminf(zmin, zv); zmax = fmaxf(zmax, zv); }
    }
    zmin = wave_min(zmin);
    zmax = wave_max(zmax);
    const int wid = threadIdx.x / TPC_WAVE, lane = threadIdx.x & (TPC_WAVE - 1);
    __syncthreads();
    if (lane == 0) { red[0][wid] = zmin; red[1][wid] = zmax; }
    __syncthreads();
    zmin = red[0][0];
    zmax = red[1][0];
    for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w) {
        zmin = fminf(zmin, red[0][w]);
        zmax = fmaxf(zmax, red[1][w]);
    }
    zlo = zmin;
    zhi = zmax;
}

// Counting sort of clusters [a, b) by cell of grid g (whole workgroup;
// contains barriers).  Writes y, z, global id in cell order to
// dy/dz/did[obase + k] and cell starts cs[c] = obase + first position of
// cell c, cs[cells] = obase + n.  cnt: LDS scratch of >= cells ints.
__device__ inline void row_sort(const float *__restrict__ y, const float *__restrict__ z, int a, int b,
                                const SegGrid &g, int *cnt, int *scan_sh, float *dy, float *dz, int32_t *did,
                                int32_t *cs, int obase) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const int cells = g.ny * g.nz;
    for (int c = tid; c < cells; c += TPC_BLOCK) cnt[c] = 0;
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        const int c = cell_coord(y[i], g.y0, g.iwy, g.ny) * g.nz + cell_coord(z[i], g.z0, g.iwz, g.nz);
        atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    // exclusive scan: each thread owns a contiguous run of cells
    const int per = (cells + TPC_BLOCK - 1) / TPC_BLOCK;
    const int c0 = tid * per;
    int c1 = c0 + per;
    if (c1 > cells) c1 = cells;
    int local = 0;
    for (int c = c0; c < c1; ++c) local += cnt[c];
    int total;
    int run = block_exclusive_scan(local, scan_sh, &total);
    for (int c = c0; c < c1; ++c) {
        const int v = cnt[c];
        cnt[c] = obase + run;         // becomes the scatter cursor
        cs[c] = obase + run;
        run += v;
    }
    if (tid == 0) cs[cells] = obase + (b - a);
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        const float yv = y[i], zv = z[i];
        const int c = cell_coord(yv, g.y0, g.iwy, g.ny) * g.nz + cell_coord(zv, g.z0, g.iwz, g.nz);
        const int slot = atomicAdd(&cnt[c], 1);
        dy[slot] = yv;
        dz[slot] = zv;
        did[slot] = i;
    }
    __syncthreads();
}

// Rows of at most this many clusters are binned in LDS by the query
// workgroup itself; an h-row with a larger neighbouring row is dense.
#define TPC_LDS_ROW 1024

__device__ inline int seg_size(const int32_t *off, int s) { return off[s + 1] - off[s]; }

// Is `seg` a non-empty interior h-row with a neighbouring row of more than
// TPC_LDS_ROW clusters (searched in slabs over the z-sorted rows)?
__device__ inline bool dense_hrow(const int32_t *off, int seg, int n_rows) {
    const int r = seg % n_rows;
    if (r == 0 || r == n_rows - 1 || seg_size(off, seg) == 0) return false;
    return seg_size(off, seg - 1) > TPC_LDS_ROW || seg_size(off, seg + 1) > TPC_LDS_ROW;
}

// Grid of a row in z alone: min(n, cap) cells of equal length over the
// finite z extent (ny = 1, so every y falls in the one cell column).
__device__ inline SegGrid zrow_grid(float zmin, float zmax, int n, int cap) {
#pragma clang fp contract(off)
    if (!(zmin <= zmax)) { zmin = 0.f; zmax = 0.f; }
    const int c = n < cap ? n : cap;
    const float rz = zmax - zmin;
    const int nz = (rz > 0.f && c > 1) ? c : 1;
    return SegGrid{0.f, zmin, 0.f, nz > 1 ? (float)nz / rz : 0.f, 1, nz, 0, 0};
}

// Counting sort of clusters [a, b) by cell of grid g through an LDS
// permutation (whole workgroup; contains barriers): the same cell order as
// row_sort, but the scatter writes 16-bit local indices into LDS and the
// sorted copy is then written in position order (coalesced stores, reads
// gathered from the row), so no partially written cache lines go to HBM.
// n = b - a <= TPC_BIN_PERM.  g has one cell column (a zrow_grid, ny = 1),
// so the cell is z's alone and y is read only by the final gather.
#ifndef TPC_BIN_PERM
#define TPC_BIN_PERM 17408   // 51 KB of LDS: three binning workgroups per CU
#endif
__device__ inline void row_sort_perm(const float *__restrict__ y, const float *__restrict__ z, int a, int b,
                                     const SegGrid &g, int *cnt, int *scan_sh, uint16_t *perm,
                                     float *__restrict__ dy, float *__restrict__ dz, int32_t *__restrict__ did,
                                     int32_t *__restrict__ cs, int obase) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const int cells = g.ny * g.nz;
    for (int c = tid; c < cells; c += TPC_BLOCK) cnt[c] = 0;
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) atomicAdd(&cnt[cell_coord(z[i], g.z0, g.iwz, g.nz)], 1);
    __syncthreads();
    const int per = (cells + TPC_BLOCK - 1) / TPC_BLOCK;
    const int c0 = tid * per;
    int c1 = c0 + per;
    if (c1 > cells) c1 = cells;
    int local = 0;
    for (int c = c0; c < c1; ++c) local += cnt[c];
    int total;
    int run = block_exclusive_scan(local, scan_sh, &total);
    for (int c = c0; c < c1; ++c) {
        const int v = cnt[c];
        cnt[c] = run;                 // becomes the scatter cursor
        cs[c] = obase + run;
        run += v;
    }
    if (tid == 0) cs[cells] = obase + (b - a);
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        const int c = cell_coord(z[i], g.z0, g.iwz, g.nz);
        perm[atomicAdd(&cnt[c], 1)] = (uint16_t)(i - a);
    }
    __syncthreads();
    // the gathers through the permutation are random within the row: z
    // first, then y, so that a workgroup's reads span one row array at a
    // time (the rows in flight on an XCD then miss its L2 less)
    for (int k = tid; k < b - a; k += TPC_BLOCK) {
        const int i = a + perm[k];
        dz[obase + k] = z[i];
        did[obase + k] = i;
    }
    __syncthreads();
    for (int k = tid; k < b - a; k += TPC_BLOCK) dy[obase + k] = y[a + perm[k]];
    __syncthreads();
}

// z-sorted global copy of segment `seg`, made only when it is a dense h-row
// or a neighbouring row of one (whole workgroup; contains barriers; L: LDS
// scratch).  With PERM the sort goes through an LDS permutation (rows of up
// to TPC_BIN_PERM clusters; larger rows scatter directly).
struct BinLds {
    int cnt[TPC_CELL_CAP];
    float red[4][TPC_BLOCK / TPC_WAVE];
    int scan_sh[TPC_BLOCK / TPC_WAVE];
};
struct BinLdsPerm : BinLds {
    uint16_t perm[TPC_BIN_PERM];
};

// Does segment `seg` need a z-sorted copy (a dense h-row or a neighbouring
// row of one)?
__device__ inline bool nb_bin_needed(const int32_t *off, int seg, int n_rows) {
    const int r = seg % n_rows;
    return dense_hrow(off, seg, n_rows) || (r >= 1 && dense_hrow(off, seg - 1, n_rows)) ||
           (r <= n_rows - 2 && dense_hrow(off, seg + 1, n_rows));
}

template <class LDS>
__device__ inline void nb_bin_seg(int seg, int n_rows, const int32_t *__restrict__ off,
                                  const float *__restrict__ y, const float *__restrict__ z, float win_y,
                                  float win_z, SegGrid *__restrict__ grid, int32_t *__restrict__ cstart,
                                  float *__restrict__ sy, float *__restrict__ sz,
                                  int32_t *__restrict__ sid, LDS &L) {
#pragma clang fp contract(off)
    int *cnt = L.cnt;
    float (*red)[TPC_BLOCK / TPC_WAVE] = L.red;
    int *scan_sh = L.scan_sh;
    if (!nb_bin_needed(off, seg, n_rows)) return;
    __syncthreads();                 // LDS reuse across calls in a persistent loop
    const int a = off[seg], b = off[seg + 1], n = b - a;
    const int base = a + seg;
    if (n == 0) {
        if (threadIdx.x == 0) {
            SegGrid g = {0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
            grid[seg] = g;
            cstart[base] = a;
        }
        return;
    }
    float zlo, zhi;
    row_zextent(z, a, b, red, zlo, zhi);
    const SegGrid g = zrow_grid(zlo, zhi, n, TPC_CELL_CAP);
    if (threadIdx.x == 0) grid[seg] = g;
    if constexpr (sizeof(LDS) >= sizeof(BinLdsPerm)) {
        if (n <= TPC_BIN_PERM) {
            row_sort_perm(y, z, a, b, g, cnt, scan_sh, L.perm, sy, sz, sid, cstart + base, a);
            return;
        }
    }
    row_sort(y, z, a, b, g, cnt, scan_sh, sy, sz, sid, cstart + base, a);
}

struct Best {
    float q;
    int32_t u, d;
};

// Lexicographic (q, u, d) order against the best so far (none yet: u < 0).
__device__ inline bool better(float q, int32_t u, int32_t d, const Best &b) {
    const bool tie = q == b.q;
    return (b.u < 0) | (q < b.q) | (tie & (u < b.u)) | (tie & (u == b.u) & (d < b.d));
}

// Best (up, down) pair for cluster (yh, zh) in the cell-sorted up row (UY,
// UZ, UI, UCS, gu) and down row (D...).  UCS[c] indexes the first cluster of
// cell c in UY/UZ/UI; a stored id k stands for cluster ubase + k (dbase + k
// in the down row).  Every operation is one single-precision rounding, and
// the predicates are evaluated on exactly the operands of the definition.
// The down row lies A rows below h and the up row B rows above (A, B in
// {1, 2}): with ay = y_u - y_h and by = y_h - y_d (z likewise) a pair passes
// |ay| <= B win, |by| <= A win and |dy| <= cut for the second difference
// dy = g (ay / B - by / A), g = 2 / (A + B), scored by q = dy*dy + dz*dz.
// At A = B = 1 every scale factor is exactly 1 and dy = ay - by, the
// adjacent-row definition; B win, ay / B and by / A are exact for the other
// distances (powers of two) and g = 2/3 is the rounded constant.
//
// Enumeration: the down-row clusters in h's window are collected first (up
// to TPC_NB_DLIST in registers); then every up-row cluster in the window is
// paired with that list.  If more down clusters are in the window, each up
// candidate instead scans the down-row cells that overlap the cut interval
// around its straight-line prediction c = h - (A / B)(u - h), of half-width
// A (A + B) / 2 cut.  Without LIST (rows dense enough that the list would
// overflow anyway) the per-up-candidate scan is used directly; the pairs
// visited, and so the result, are the same.  Cells scanned are those
// overlapping the window (or
// cut) interval widened by a margin m far above the rounding of the
// predicates and of c; as cell_coord is monotonic, every cluster that can
// pass the exact predicates is visited.  A cluster h with a non-finite
// coordinate fails every window, so it is skipped.
#define TPC_NB_DLIST 8

template <int A = 1, int B = 1, bool LIST = true, class FP, class IP, class CP>
__device__ inline Best best_pair(float yh, float zh, FP UY, FP UZ, IP UI, CP UCS, const SegGrid &gu,
                                 int32_t ubase, FP DY, FP DZ, IP DI, CP DCS, const SegGrid &gd,
                                 int32_t dbase, float win_y, float win_z, float cut_y, float cut_z) {
#pragma clang fp contract(off)
    static_assert(A >= 1 && A <= 2 && B >= 1 && B <= 2, "partners one or two rows away");
    constexpr float fa = (float)A, fb = (float)B;
    constexpr float g = 2.0f / (float)(A + B);
    constexpr float kw = A > B ? fa : fb;              // widest window, in windows
    constexpr float kc = (float)(A * (A + B)) / 2.0f;  // cut interval of the down row, in cuts
    constexpr float rab = fa / fb;                     // prediction slope of the down row
    Best best = {0.f, -1, -1};
    if (gu.ny <= 0 || gd.ny <= 0 || !isfinite(yh) || !isfinite(zh)) return best;
    const float my = 1e-5f * (fabsf(yh) + kw * win_y + kc * cut_y) + 1e-6f;
    const float mz = 1e-5f * (fabsf(zh) + kw * win_z + kc * cut_z) + 1e-6f;
    const float wdy = fa * win_y + my, wdz = fa * win_z + mz;
    const float wuy = fb * win_y + my, wuz = fb * win_z + mz;
    const float ky = kc * cut_y + my, kz = kc * cut_z + mz;
    // down clusters in the window (by / A kept)
    float lb[TPC_NB_DLIST][2];
    int32_t ld[TPC_NB_DLIST];
#pragma unroll
    for (int j = 0; j < TPC_NB_DLIST; ++j) { lb[j][0] = 0.f; lb[j][1] = 0.f; ld[j] = -1; }
    int nd = 0;
    if constexpr (LIST) {
        const int y0 = cell_coord(yh - wdy, gd.y0, gd.iwy, gd.ny), y1 = cell_coord(yh + wdy, gd.y0, gd.iwy, gd.ny);
        const int z0 = cell_coord(zh - wdz, gd.z0, gd.iwz, gd.nz), z1 = cell_coord(zh + wdz, gd.z0, gd.iwz, gd.nz);
        for (int iy = y0; iy <= y1; ++iy) {
            const int e0 = DCS[iy * gd.nz + z0];
            const int e1 = DCS[iy * gd.nz + z1 + 1];
            for (int kd = e0; kd < e1; ++kd) {
                const float by = yh - DY[kd];
                const float bz = zh - DZ[kd];
                if (!(fabsf(by) <= fa * win_y && fabsf(bz) <= fa * win_z)) continue;
                const int32_t d = dbase + (int32_t)DI[kd];
                const float sy = by / fa, sz = bz / fa;
#pragma unroll
                for (int j = 0; j < TPC_NB_DLIST; ++j)
                    if (nd == j) { lb[j][0] = sy; lb[j][1] = sz; ld[j] = d; }
                ++nd;
            }
        }
    }
    if (LIST && nd == 0) return best;
    const bool listed = LIST && nd <= TPC_NB_DLIST;
    const int yu0 = cell_coord(yh - wuy, gu.y0, gu.iwy, gu.ny), yu1 = cell_coord(yh + wuy, gu.y0, gu.iwy, gu.ny);
    const int zu0 = cell_coord(zh - wuz, gu.z0, gu.iwz, gu.nz), zu1 = cell_coord(zh + wuz, gu.z0, gu.iwz, gu.nz);
    for (int iyu = yu0; iyu <= yu1; ++iyu) {
        const int ue0 = UCS[iyu * gu.nz + zu0];
        const int ue1 = UCS[iyu * gu.nz + zu1 + 1];
        for (int ku = ue0; ku < ue1; ++ku) {
            const float ay = UY[ku] - yh;
            const float az = UZ[ku] - zh;
            if (!(fabsf(ay) <= fb * win_y && fabsf(az) <= fb * win_z)) continue;
            const int32_t u = ubase + (int32_t)UI[ku];
            const float ty = ay / fb, tz = az / fb;
            if (listed) {
#pragma unroll
                for (int j = 0; j < TPC_NB_DLIST; ++j) {
                    const float ey = ty - lb[j][0];
                    const float ez = tz - lb[j][1];
                    const float dy = g * ey;
                    const float dz = g * ez;
                    if (j < nd && fabsf(dy) <= cut_y && fabsf(dz) <= cut_z) {
                        const float qy = dy * dy;
                        const float qz = dz * dz;
                        const float q = qy + qz;
                        if (better(q, u, ld[j], best)) { best.q = q; best.u = u; best.d = ld[j]; }
                    }
                }
                continue;
            }
            const float cy = yh - rab * ay, cz = zh - rab * az;
            const int yd0 = cell_coord(cy - ky, gd.y0, gd.iwy, gd.ny);
            const int yd1 = cell_coord(cy + ky, gd.y0, gd.iwy, gd.ny);
            const int zd0 = cell_coord(cz - kz, gd.z0, gd.iwz, gd.nz);
            const int zd1 = cell_coord(cz + kz, gd.z0, gd.iwz, gd.nz);
            for (int iyd = yd0; iyd <= yd1; ++iyd) {
                const int de0 = DCS[iyd * gd.nz + zd0];
                const int de1 = DCS[iyd * gd.nz + zd1 + 1];
                for (int kd = de0; kd < de1; ++kd) {
                    const float by = yh - DY[kd];
                    const float bz = zh - DZ[kd];
                    if (!(fabsf(by) <= fa * win_y && fabsf(bz) <= fa * win_z)) continue;
                    const float ey = ty - by / fa;
                    const float ez = tz - bz / fa;
                    const float dy = g * ey;
                    const float dz = g * ez;
                    if (!(fabsf(dy) <= cut_y && fabsf(dz) <= cut_z)) continue;
                    const float qy = dy * dy;
                    const float qz = dz * dz;
                    const float q = qy + qz;
                    const int32_t d = dbase + (int32_t)DI[kd];
                    if (better(q, u, d, best)) { best.q = q; best.u = u; best.d = d; }
                }
            }
        }
    }
    return best;
}

// LDS form of a row pair: both rows of up to ROW clusters each, with finer
// cells than the global form (up to 4 per cluster, CELLS per row) so that
// the cells around h hold few candidates.  Two sizes: the small one keeps
// the workgroup's LDS at 18 KB (8 workgroups per CU), the large one at
// 37 KB for rows of up to TPC_LDS_ROW clusters.
#ifndef TPC_LDS_CELLS
#define TPC_LDS_CELLS 2048
#endif
#define TPC_LDS_ROW_S 512
#define TPC_LDS_CELLS_S 1024

template <int ROW, int CELLS>
struct PairLdsT {
    float y[2 * ROW], z[2 * ROW];
    uint16_t rel[2 * ROW];                  // cluster id minus its row's first id
    int32_t cs[2 * CELLS + 2];              // cell starts of both rows, concatenated
    float red[8][TPC_BLOCK / TPC_WAVE];
    int scan_sh[TPC_BLOCK / TPC_WAVE];
};
using PairLds = PairLdsT<TPC_LDS_ROW, TPC_LDS_CELLS>;
using PairLdsSmall = PairLdsT<TPC_LDS_ROW_S, TPC_LDS_CELLS_S>;

// Bins a down row of n0 clusters and an up row of n1 clusters with one LDS
// counting sort over the concatenated cell range (whole workgroup; contains
// barriers).  src(k, y, z, rel) gives cluster k of the pair (the down row
// first) and its id relative to its row's first cluster.  On return the
// down row occupies cells [0, C0) with grid gd, the up row cells C0 + [0, C1)
// with grid gu, and cell c holds positions [cs[c], cs[c+1]) of y/z/rel.
// Cell edges are at least edge_d (down row) and edge_u (up row) windows.
__device__ inline int pair_cell(float yv, float zv, const SegGrid &g) {
    return cell_coord(yv, g.y0, g.iwy, g.ny) * g.nz + cell_coord(zv, g.z0, g.iwz, g.nz);
}

template <int CELLS>
__device__ inline SegGrid pair_grid(float ymin, float ymax, float zmin, float zmax, int n, float win_y,
                                    float win_z, float edge) {
    if (n == 0) return SegGrid{0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
    const int cap = 4 * n < CELLS ? 4 * n : CELLS;
    return row_grid(ymin, ymax, zmin, zmax, cap, cap, win_y, win_z, edge);
}

// The clusters of two row ranges of the frame arrays: [ra0, ra0 + n0), then
// [ra1, ...); relative ids are the offsets in the range.
struct RowPairSrc {
    const float *y, *z;
    int ra0, n0, ra1;
    __device__ void operator()(int k, float &vy, float &vz, uint16_t &rel) const {
        const int i = k < n0 ? ra0 + k : ra1 + (k - n0);
        vy = y[i];
        vz = z[i];
        rel = (uint16_t)(k < n0 ? k : k - n0);
    }
};

// Two position ranges of the z-sorted copies (sy, sz, sid): [pa0, pa0 + n0)
// of the down row, whose first cluster id is base0, then [pa1, ...) of the
// up row (base1).
struct SortedPairSrc {
    const float *sy, *sz;
    const int32_t *sid;
    int pa0, n0, pa1, base0, base1;
    __device__ void operator()(int k, float &vy, float &vz, uint16_t &rel) const {
        const int p = k < n0 ? pa0 + k : pa1 + (k - n0);
        vy = sy[p];
        vz = sz[p];
        rel = (uint16_t)(sid[p] - (k < n0 ? base0 : base1));
    }
};

template <int ROW, int CELLS, class Src>
__device__ inline void pair_bin(const Src &src, int n0, int n1, float win_y, float win_z, float edge_d,
                                float edge_u,
                                PairLdsT<ROW, CELLS> &L, SegGrid &gd, SegGrid &gu, int &C0) {
#pragma clang fp contract(off)
    constexpr int PT = 2 * ROW / TPC_BLOCK;      // row-pair clusters per thread
    const int tid = threadIdx.x;
    const int nt = n0 + n1;
    // both rows are read once, into registers (one global round trip)
    float vy[PT], vz[PT];
    uint16_t vr[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int k = tid + j * TPC_BLOCK;
        vy[j] = 0.f;
        vz[j] = 0.f;
        vr[j] = 0;
        if (k < nt) src(k, vy[j], vz[j], vr[j]);
    }
    // finite extents of both rows
    float e[8] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int k = tid + j * TPC_BLOCK;
        const bool fy = k < nt && isfinite(vy[j]), fz = k < nt && isfinite(vz[j]);
        if (k < n0) {
            if (fy) { e[0] = fminf(e[0], vy[j]); e[1] = fmaxf(e[1], vy[j]); }
            if (fz) { e[2] = fminf(e[2], vz[j]); e[3] = fmaxf(e[3], vz[j]); }
        } else {
            if (fy) { e[4] = fminf(e[4], vy[j]); e[5] = fmaxf(e[5], vy[j]); }
            if (fz) { e[6] = fminf(e[6], vz[j]); e[7] = fmaxf(e[7], vz[j]); }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = (j & 1) ? wave_max(e[j]) : wave_min(e[j]);
    const int wid = tid / TPC_WAVE, lane = tid & (TPC_WAVE - 1);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) L.red[j][wid] = e[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float v = L.red[j][0];
#pragma unroll
        for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w)
            v = (j & 1) ? fmaxf(v, L.red[j][w]) : fminf(v, L.red[j][w]);
        e[j] = v;
    }
    gd = pair_grid<CELLS>(e[0], e[1], e[2], e[3], n0, win_y, win_z, edge_d);
    gu = pair_grid<CELLS>(e[4], e[5], e[6], e[7], n1, win_y, win_z, edge_u);
    C0 = gd.ny * gd.nz;
    const int C = C0 + gu.ny * gu.nz;
    for (int c = tid; c < C + 2; c += TPC_BLOCK) L.cs[c] = 0;
    __syncthreads();
    // count cell c into cs[c + 2]
    int cell[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int k = tid + j * TPC_BLOCK;
        cell[j] = k < n0 ? pair_cell(vy[j], vz[j], gd) : C0 + pair_cell(vy[j], vz[j], gu);
        if (k < nt) atomicAdd(&L.cs[cell[j] + 2], 1);
    }
    __syncthreads();
    // inclusive scan of cs[1 .. C+1] (cs[1] is 0): cs[c + 1] = first position of cell c
    const int len = C + 1;
    const int per = (len + TPC_BLOCK - 1) / TPC_BLOCK;
    const int j0 = 1 + tid * per;
    const int j1 = j0 + per < 1 + len ? j0 + per : 1 + len;
    int local = 0;
    for (int j = j0; j < j1; ++j) local += L.cs[j];
    int total;
    int run = block_exclusive_scan(local, L.scan_sh, &total);
    for (int j = j0; j < j1; ++j) {
        run += L.cs[j];
        L.cs[j] = run;
    }
    __syncthreads();
    // scatter; the cursor of cell c moves from its start to its end, which
    // leaves cs[c] = start of cell c for every c in [0, C]
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int k = tid + j * TPC_BLOCK;
        if (k < nt) {
            const int slot = atomicAdd(&L.cs[cell[j] + 1], 1);
            L.y[slot] = vy[j];
            L.z[slot] = vz[j];
            L.rel[slot] = vr[j];
        }
    }
    __syncthreads();
}

// Does h-row `seg` (an interior, non-empty row) have neighbour rows that fit
// the small LDS form?
__device__ inline bool small_pair(const int32_t *off, int seg) {
    return seg_size(off, seg - 1) <= TPC_LDS_ROW_S && seg_size(off, seg + 1) <= TPC_LDS_ROW_S;
}

// Which segments a query call handles: rows whose neighbour rows fit the
// small LDS form, the other rows whose neighbour rows fit the large form,
// both, or the dense rows (a neighbour row of more than TPC_LDS_ROW).
enum NbClass { NB_NOT_DENSE = 0, NB_SMALL = 1, NB_LARGE = 2, NB_DENSE = 3 };

// Tunables of the dense-row search: h clusters per slab (the slab's
// clusters are consecutive in the z-sorted h-row), the smallest slab before
// the global fallback, the row-pair LDS size of a slab, and the LDS cell
// edges of a slab's down and up rows in windows (the down row is only
// searched around predictions, in boxes of twice the cuts; the up row in
// windows).
#ifndef TPC_NB_SLAB
#define TPC_NB_SLAB 512
#endif
#ifndef TPC_NB_SLAB_MIN
#define TPC_NB_SLAB_MIN 64
#endif
#ifndef TPC_NB_DENSE_ROW
#define TPC_NB_DENSE_ROW 1024
#endif
#ifndef TPC_NB_DENSE_CELLS
#define TPC_NB_DENSE_CELLS 2048
#endif
#ifndef TPC_NB_DENSE_EDGE_D
#define TPC_NB_DENSE_EDGE_D 0.18f
#endif
#ifndef TPC_NB_DENSE_EDGE_U
#define TPC_NB_DENSE_EDGE_U 0.25f
#endif
// LDS of a dense-row workgroup: the slab's row pair and the slab's results
// (up id << 16 | down id relative to their rows, all ones for none), which
// are written out once the slab is searched.
template <int ROW, int CELLS>
struct DenseLdsT : PairLdsT<ROW, CELLS> {
    uint32_t res[TPC_NB_SLAB];
};
using DenseLds = DenseLdsT<TPC_NB_DENSE_ROW, TPC_NB_DENSE_CELLS>;

// Positions [x, y) of the z-sorted copy of a row (grid g, cell starts cs)
// that hold every cluster with z in [lo, hi] (whole cells: cell_coord is
// monotonic, so a cluster with z in the interval lies in a cell between
// those of lo and hi).
__device__ inline int2 zrange(const SegGrid &g, const int32_t *cs, float lo, float hi) {
    if (g.ny <= 0) return make_int2(0, 0);
    const int c0 = cell_coord(lo, g.z0, g.iwz, g.nz), c1 = cell_coord(hi, g.z0, g.iwz, g.nz);
    return make_int2(cs[c0], cs[c1 + 1]);
}

// Search of one slab (clusters [pb, pb + pn) of the h-row's z-sorted copy)
// whose row pair is binned in L (whole workgroup): the result of
// best_pair<1, 1> for every cluster h, by the same single-precision
// operations on a pruned set of candidates.  A lane takes clusters h of the
// slab in turn (consecutive lanes, consecutive positions: nearby z) and walks
// the up-row cells of h's window; for every u in the window it scans the
// down-row cells of the box around the prediction 2h - u.  Once a passing
// triplet of score q* is known the box half-widths shrink from the cuts to
// sqrt(q*) (1 + 1e-4) plus the rounding margin: a down cluster outside has
// |dy| or |dz| above sqrt(q*), so fl(dy^2) + fl(dz^2) > q* (rounding is
// monotonic and both squares are >= 0) and it can neither beat nor tie the
// best, whose lexicographic order (q, then u id, then d id) is kept
// exactly.
//
// The nested walks of one cluster (up-row window cells, their candidates,
// and for each up cluster in the window the down-row box cells and their
// candidates) run as one flat loop in which every iteration tests one LDS
// candidate per lane, so lanes at different depths of the walk stay in
// step; a lane moves to its next cluster (every TPC_BLOCK-th of the slab,
// loaded while it searches the current one) when the current one is
// exhausted.  One candidate test serves both walks: a candidate c at
// (t_y, t_z) = (y_c - y_h, z_c - z_h) passes the window test on |t| in
// either; an up candidate then starts a down box, a down candidate is
// scored with d_y = a_y + t_y, equal (rounding included) to
// a_y - (y_h - y_d) since fl(y_h - y_d) = -fl(y_d - y_h).  The best so far
// is one 64-bit key (bits of q, then the up and down ids, 16 bits each), so
// the lexicographic order is one unsigned comparison (q >= 0, whose bit
// patterns order as its values) and the test carries no branches.
//
// Cell ranges are computed in cell units: the window's or the prediction's
// cell coordinate is (y_h - y0) iw (minus a_y iw for the prediction), its
// half-width (w + m) iw plus e = 1e-6 (|y0| iw + 1) cells, where w is the
// window or min(cut, sqrt(q*) (1 + 1e-4)).  These products round
// differently from cell_coord at the range's edge by a few units of 2^-24
// of (|y_h| + |y0| + w) iw, which m (1e-5 of |y_h| + window + cut) and e
// cover, so every cluster that can pass lies in the cells scanned.  The
// square root of the box set-up is the hardware estimate (a few ulp at
// most; a denormal q* may give 0, which only shrinks the box to its
// rounding margin, still far above sqrt(q*)): the 1e-4 widening covers it.
__device__ inline int cell_in(float c, float nmax) { return (int)__builtin_amdgcn_fmed3f(c, 0.0f, nmax); }

template <int ROW, int CELLS>
__device__ inline void slab_search(int pb, int pn, const float *__restrict__ sy, const float *__restrict__ sz,
                                   const int32_t *__restrict__ sid, int32_t baseu, int32_t based,
                                   const SegGrid &gu, const SegGrid &gd, int C0, float win_y, float win_z,
                                   float cut_y, float cut_z, int32_t *__restrict__ up,
                                   int32_t *__restrict__ dn, DenseLdsT<ROW, CELLS> &L) {
#pragma clang fp contract(off)
    const float *Y = L.y, *Z = L.z;
    const uint16_t *R = L.rel;
    const int32_t *UCS = L.cs + C0, *DCS = L.cs;
    const bool grids = gu.ny > 0 && gd.ny > 0;
    constexpr uint64_t NONE = (0x7F800000ull << 32) | 0xFFFFFFFFull;
    const float edy = 1e-6f * (fabsf(gd.y0) * gd.iwy + 1.0f), edz = 1e-6f * (fabsf(gd.z0) * gd.iwz + 1.0f);
    const float euy = 1e-6f * (fabsf(gu.y0) * gu.iwy + 1.0f), euz = 1e-6f * (fabsf(gu.z0) * gu.iwz + 1.0f);
    const float dny = (float)(gd.ny - 1), dnz = (float)(gd.nz - 1);
    const float uny = (float)(gu.ny - 1), unz = (float)(gu.nz - 1);
    const float wcy = win_y + cut_y, wcz = win_z + cut_z;
    int j = (int)threadIdx.x - TPC_BLOCK;
    bool active = false, dmode = false;
    float yh = 0.f, zh = 0.f, hy = 0.f, hz = 0.f, my = 0.f, mz = 0.f, ay = 0.f, az = 0.f;
    float yn = 0.f, zn = 0.f;
    if ((int)threadIdx.x < pn) {
        yn = sy[pb + threadIdx.x];
        zn = sz[pb + threadIdx.x];
    }
    uint64_t best = NONE;
    uint32_t urs = 0;
    int iy = 0, iy1 = -1, zc0 = 0, zc1 = 0, k = 0, k1 = 0;
    int yd = 0, yd1 = -1, zd0 = 0, zd1 = 0, kd = 0, e1 = 0;
    while (true) {
        if (!active) {
            j += TPC_BLOCK;
            if (j < pn) {
                yh = yn;
                zh = zn;
                if (j + TPC_BLOCK < pn) {
                    yn = sy[pb + j + TPC_BLOCK];
                    zn = sz[pb + j + TPC_BLOCK];
                }
                best = NONE;
                dmode = false;
                iy = 0; iy1 = -1; k = 0; k1 = 0;
                if (grids && isfinite(yh) && isfinite(zh)) {
                    my = __builtin_fmaf(fabsf(yh) + wcy, 1e-5f, 1e-6f);
                    mz = __builtin_fmaf(fabsf(zh) + wcz, 1e-5f, 1e-6f);
                    hy = (yh - gd.y0) * gd.iwy;
                    hz = (zh - gd.z0) * gd.iwz;
                    const float uy = (yh - gu.y0) * gu.iwy, uz = (zh - gu.z0) * gu.iwz;
                    const float wy = __builtin_fmaf(win_y + my, gu.iwy, euy);
                    const float wz = __builtin_fmaf(win_z + mz, gu.iwz, euz);
                    iy = cell_in(uy - wy, uny);
                    iy1 = cell_in(uy + wy, uny);
                    zc0 = cell_in(uz - wz, unz);
                    zc1 = cell_in(uz + wz, unz);
                    const int row = __mul24(iy, gu.nz);
                    k = UCS[row + zc0];
                    k1 = UCS[row + zc1 + 1];
                }
                active = true;
            }
        }
        if (__ballot(active) == 0ull) break;
        if (!active) continue;
        if (dmode) {
            while (kd == e1 && yd < yd1) {
                ++yd;
                kd = DCS[yd * gd.nz + zd0];
                e1 = DCS[yd * gd.nz + zd1 + 1];
            }
            dmode = kd < e1;
        }
        if (!dmode) {
            while (k == k1 && iy < iy1) {
                ++iy;
                k = UCS[iy * gu.nz + zc0];
                k1 = UCS[iy * gu.nz + zc1 + 1];
            }
            if (k == k1) {                            // cluster done
                L.res[j] = best != NONE ? (uint32_t)best : 0xFFFFFFFFu;
                active = false;
                continue;
            }
        }
        const int c = dmode ? kd : k;
        kd += (int)dmode;
        k += (int)!dmode;
        const float ty = Y[c] - yh;
        const float tz = Z[c] - zh;
        const uint32_t rr = R[c];
        // bitwise, not short-circuit, conjunctions: no branches in the test
        const bool inwin = (int)(fabsf(ty) <= win_y) & (int)(fabsf(tz) <= win_z);
        const float dy = ay + ty;
        const float dz = az + tz;
        const float qy = dy * dy;
        const float qz = dz * dz;
        const float q = qy + qz;
        const uint64_t key = ((uint64_t)__float_as_uint(q) << 32) | (uint64_t)(urs | rr);
        const bool win = (int)dmode & (int)inwin & (int)(fabsf(dy) <= cut_y) & (int)(fabsf(dz) <= cut_z) &
                         (int)(key < best);
        best = win ? key : best;
        if (!dmode && inwin) {
            // down clusters around the prediction h - (u - h)
            ay = ty;
            az = tz;
            urs = rr << 16;
            const float r = __builtin_amdgcn_sqrtf(__uint_as_float((uint32_t)(best >> 32))) * 1.0001f;
            const float py = __builtin_fmaf(-ty, gd.iwy, hy), pz = __builtin_fmaf(-tz, gd.iwz, hz);
            const float ky = __builtin_fmaf(fminf(cut_y, r) + my, gd.iwy, edy);
            const float kz = __builtin_fmaf(fminf(cut_z, r) + mz, gd.iwz, edz);
            yd = cell_in(py - ky, dny);
            yd1 = cell_in(py + ky, dny);
            zd0 = cell_in(pz - kz, dnz);
            zd1 = cell_in(pz + kz, dnz);
            const int row = __mul24(yd, gd.nz);
            kd = DCS[row + zd0];
            e1 = DCS[row + zd1 + 1];
            dmode = true;
        }
    }
    // results in the slab's order (ids read coalesced; the search loop
    // issues no global store, whose completion its waits for the next
    // cluster's loads would also wait for)
    __syncthreads();
    for (int p = threadIdx.x; p < pn; p += TPC_BLOCK) {
        const uint32_t r = L.res[p];
        const int32_t h = sid[pb + p];
        up[h] = r == 0xFFFFFFFFu ? -1 : baseu + (int32_t)(r >> 16);
        dn[h] = r == 0xFFFFFFFFu ? -1 : based + (int32_t)(r & 0xFFFFu);
    }
}

// Start of part k of a dense h-row of n z-sorted clusters searched in
// `parts` parts by different workgroups: k / parts of it, rounded down to
// whole slabs (part parts ends at n).
__device__ inline int dense_split(int n, int k, int parts) {
    return k >= parts ? n : (int)((int64_t)n * k / parts) / TPC_NB_SLAB * TPC_NB_SLAB;
}

// Dense h-row `seg` (whole workgroup; contains barriers): slabs of
// consecutive clusters of its z-sorted copy.  A partner of h passes the
// window test only if its z lies within win_z of z_h (the difference is one
// rounding), so the neighbouring rows' clusters with z in the slab's finite
// z extent widened by win_z and a margin far above that rounding hold every
// candidate; their positions form one range of each z-sorted copy.  Both
// ranges are binned into LDS and the slab searched there (slab_search); a
// slab whose ranges do not fit is halved, and at TPC_NB_SLAB_MIN clusters it
// is searched in the global copies instead.  The outcome does not depend
// on which superset of the candidates is searched.
template <int ROW, int CELLS>
__device__ inline void nb_dense_seg(int seg, const int32_t *__restrict__ off, int32_t n_rows, float win_y,
                                    float win_z, float cut_y, float cut_z, const SegGrid *__restrict__ grid,
                                    const int32_t *__restrict__ cstart, const float *__restrict__ sy,
                                    const float *__restrict__ sz, const int32_t *__restrict__ sid,
                                    int32_t *__restrict__ up, int32_t *__restrict__ dn,
                                    DenseLdsT<ROW, CELLS> &L, int part = 0, int parts = 1) {
#pragma clang fp contract(off)
    if (!dense_hrow(off, seg, n_rows)) return;
    const int tid = threadIdx.x;
    const int a = off[seg], n = off[seg + 1] - a;
    const int lo = dense_split(n, part, parts), hi = dense_split(n, part + 1, parts);
    const int sd = seg - 1, su = seg + 1;
    const int based = off[sd], baseu = off[su];
    const SegGrid gdg = grid[sd], gug = grid[su];
    const int32_t *csd = cstart + based + sd;
    const int32_t *csu = cstart + baseu + su;
    // relative ids are 16-bit in the keys and in LDS (at most 65534, so a
    // result is never all ones)
    const bool rel_ok = seg_size(off, sd) <= 65535 && seg_size(off, su) <= 65535;
    int P = TPC_NB_SLAB;
    for (int p0 = lo; p0 < hi;) {
        const int pn = hi - p0 < P ? hi - p0 : P;
        float lo = INFINITY, hi = -INFINITY;
        for (int k = tid; k < pn; k += TPC_BLOCK) {
            const float zv = sz[a + p0 + k];
            if (isfinite(zv)) { lo = fminf(lo, zv); hi = fmaxf(hi, zv); }
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        __syncthreads();             // the previous slab's search is done with L
        if ((tid & (TPC_WAVE - 1)) == 0) {
            L.red[0][tid / TPC_WAVE] = lo;
            L.red[1][tid / TPC_WAVE] = hi;
        }
        __syncthreads();
        lo = L.red[0][0];
        hi = L.red[1][0];
        for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w) {
            lo = fminf(lo, L.red[0][w]);
            hi = fmaxf(hi, L.red[1][w]);
        }
        __syncthreads();             // everyone has read L.red
        int2 rd = make_int2(0, 0), ru = make_int2(0, 0);
        if (lo <= hi) {
            const float m = 1e-5f * (fmaxf(fabsf(lo), fabsf(hi)) + win_z + cut_z) + 1e-6f;
            const float w = win_z + m;
            rd = zrange(gdg, csd, lo - w, hi + w);
            ru = zrange(gug, csu, lo - w, hi + w);
        }
        const int nd = rd.y - rd.x, nu = ru.y - ru.x;
        const bool fits = rel_ok && nd <= ROW && nu <= ROW;
        if (!fits && P > TPC_NB_SLAB_MIN) {
            P >>= 1;
            continue;
        }
        if (fits) {
            SegGrid gd, gu;
            int C0;
            pair_bin(SortedPairSrc{sy, sz, sid, rd.x, nd, ru.x, based, baseu}, nd, nu, win_y, win_z,
                     TPC_NB_DENSE_EDGE_D, TPC_NB_DENSE_EDGE_U, L, gd, gu, C0);
            slab_search(a + p0, pn, sy, sz, sid, baseu, based, gu, gd, C0, win_y, win_z, cut_y, cut_z, up, dn,
                        L);
        } else {
            for (int k = tid; k < pn; k += TPC_BLOCK) {
                const int p = a + p0 + k;
                const Best bt = best_pair(sy[p], sz[p], sy, sz, sid, csu, gug, 0, sy, sz, sid, csd, gdg, 0,
                                          win_y, win_z, cut_y, cut_z);
                const int32_t h = sid[p];
                up[h] = bt.u;
                dn[h] = bt.d;
            }
        }
        p0 += pn;
        P = TPC_NB_SLAB;
    }
    __syncthreads();                 // LDS reuse across calls in a persistent loop
}

// Best triplet of every cluster of h-row `seg` (whole workgroup; contains
// barriers; L is the workgroup's LDS scratch).  When both neighbouring rows
// hold at most ROW clusters the workgroup bins them itself into LDS
// (coalesced reads, then every candidate access is an LDS access);
// dense rows are left to nb_dense_seg.  cls selects the segments handled
// (the others return at once), so that a small-LDS and a large-LDS launch
// can share the rows between them.
template <int ROW, int CELLS>
__device__ inline void nb_query_seg(int seg, const int32_t *__restrict__ off, int32_t n_rows,
                                    const float *__restrict__ y, const float *__restrict__ z,
                                    float win_y, float win_z, float cut_y, float cut_z,
                                    const SegGrid *__restrict__ grid, const int32_t *__restrict__ cstart,
                                    const float *__restrict__ sy, const float *__restrict__ sz,
                                    const int32_t *__restrict__ sid, int32_t *__restrict__ up,
                                    int32_t *__restrict__ dn, PairLdsT<ROW, CELLS> &L, NbClass cls) {
#pragma clang fp contract(off)
    static_assert(ROW == TPC_LDS_ROW || ROW == TPC_LDS_ROW_S, "row-pair LDS forms");
    const int r = seg % n_rows;
    const int a = off[seg], b = off[seg + 1];
    const bool edge = r == 0 || r == n_rows - 1;
    const bool small = !edge && a != b && small_pair(off, seg);
    if ((cls == NB_SMALL && !small) || (cls == NB_LARGE && small)) return;
    if (dense_hrow(off, seg, n_rows)) return;
    if (edge) {
        for (int i = a + threadIdx.x; i < b; i += TPC_BLOCK) { up[i] = -1; dn[i] = -1; }
        return;
    }
    if (a == b) return;
    if (seg_size(off, seg - 1) <= ROW && seg_size(off, seg + 1) <= ROW) {
        const int ra0 = off[seg - 1], ra1 = off[seg + 1];
        // the first h of each thread is loaded together with the row pair
        float hy = 0.f, hz = 0.f;
        if (a + (int)threadIdx.x < b) {
            hy = y[a + threadIdx.x];
            hz = z[a + threadIdx.x];
        }
        SegGrid gd, gu;
        int C0;
        pair_bin(RowPairSrc{y, z, ra0, a - ra0, ra1}, a - ra0, off[seg + 2] - ra1, win_y, win_z, 1.01f,
                 1.01f, L, gd, gu, C0);
        for (int i = a + threadIdx.x; i < b; i += TPC_BLOCK) {
            if (i >= a + TPC_BLOCK) {
                hy = y[i];
                hz = z[i];
            }
            const Best bt = best_pair(hy, hz, L.y, L.z, L.rel, L.cs + C0, gu, ra1, L.y, L.z, L.rel,
                                      L.cs, gd, ra0, win_y, win_z, cut_y, cut_z);
            up[i] = bt.u;
            dn[i] = bt.d;
        }
        __syncthreads();             // LDS reuse across calls in a persistent loop
        return;
    }
}

}  // namespace tpc_nb
