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
// Design: two passes, one workgroup per (frame, sector, row) segment.
//  1. nb_bin: per segment, a y-z cell grid sized from the data (cell edges at
//     least 1.01 x the window, at most one cell per cluster, at most
//     TPC_CELL_CAP cells); an LDS counting sort writes the segment's clusters
//     cell by cell (coalesced SoA y, z, id) and the cell start table.
//  2. nb_query: each thread takes one cluster h in cell order, so a wavefront
//     walks neighbouring cells of rows r+1 and r-1 together; for each
//     candidate the window/cut predicates are evaluated exactly as defined.
// Candidates with |y_u - y_h| <= win differ by at most one cell because the
// cell edge exceeds the window by 1%, far more than the rounding of the cell
// coordinate, and clamping keeps that bound; so scanning the 3x3 cells
// around h over-covers the window and the exact predicates decide.
#include "tpc_internal.hpp"

namespace tpc_nb {


__device__ inline int cell_coord(float v, float v0, float iw, int n) {
#pragma clang fp contract(off)
    if (n <= 1) return 0;
    float c = (v - v0) * iw;
    if (!(c >= 0.0f)) return 0;                     // negative or NaN
    if (c >= (float)(n - 1)) return n - 1;          // also +inf
    return (int)c;                                  // floor for c >= 0
}

// Bins the clusters of segment `seg` (whole workgroup; contains barriers).
__device__ inline void nb_bin_seg(int seg, const int32_t *__restrict__ off, const float *__restrict__ y,
                                  const float *__restrict__ z, float win_y, float win_z,
                                  SegGrid *__restrict__ grid, int32_t *__restrict__ cstart,
                                  float *__restrict__ sy, float *__restrict__ sz,
                                  int32_t *__restrict__ sid) {
#pragma clang fp contract(off)
    __shared__ int cnt[TPC_CELL_CAP];
    __shared__ float red[4][TPC_BLOCK / TPC_WAVE];
    __shared__ int scan_sh[TPC_BLOCK / TPC_WAVE];
    __syncthreads();                 // LDS reuse across calls in a persistent loop
    const int a = off[seg], b = off[seg + 1], n = b - a;
    const int base = a + seg;
    const int tid = threadIdx.x;
    if (n == 0) {
        if (tid == 0) {
            SegGrid g = {0.f, 0.f, 0.f, 0.f, 0, 0, 0, 0};
            grid[seg] = g;
            cstart[base] = a;
        }
        return;
    }
    // finite extent of the segment
    float ymin = INFINITY, ymax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        float yv = y[i], zv = z[i];
        if (isfinite(yv)) { ymin = fminf(ymin, yv); ymax = fmaxf(ymax, yv); }
        if (isfinite(zv)) { zmin = fminf(zmin, zv); zmax = fmaxf(zmax, zv); }
    }
    ymin = wave_min(ymin); ymax = wave_max(ymax);
    zmin = wave_min(zmin); zmax = wave_max(zmax);
    const int wid = tid / TPC_WAVE, lane = tid & (TPC_WAVE - 1);
    if (lane == 0) { red[0][wid] = ymin; red[1][wid] = ymax; red[2][wid] = zmin; red[3][wid] = zmax; }
    __syncthreads();
    ymin = red[0][0]; ymax = red[1][0]; zmin = red[2][0]; zmax = red[3][0];
    for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w) {
        ymin = fminf(ymin, red[0][w]); ymax = fmaxf(ymax, red[1][w]);
        zmin = fminf(zmin, red[2][w]); zmax = fmaxf(zmax, red[3][w]);
    }
    if (!(ymin <= ymax)) { ymin = 0.f; ymax = 0.f; }
    if (!(zmin <= zmax)) { zmin = 0.f; zmax = 0.f; }
    // cell counts: edges >= 1.01 * window, cells <= min(n, cap)
    const int cap = n < TPC_CELL_CAP ? n : TPC_CELL_CAP;
    const float ry = ymax - ymin, rz = zmax - zmin;
    float fz = rz / (1.01f * win_z), fy = ry / (1.01f * win_y);
    int nzmax = fz >= (float)cap ? cap : (fz >= 1.0f ? (int)fz : 1);
    int nymax = fy >= (float)cap ? cap : (fy >= 1.0f ? (int)fy : 1);
    int nz = nzmax;
    int ny = cap / nz;
    if (ny > nymax) ny = nymax;
    if (ny < 1) ny = 1;
    const float iwy = ny > 1 ? (float)ny / ry : 0.f;
    const float iwz = nz > 1 ? (float)nz / rz : 0.f;
    const int cells = ny * nz;
    for (int c = tid; c < cells; c += TPC_BLOCK) cnt[c] = 0;
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        int c = cell_coord(y[i], ymin, iwy, ny) * nz + cell_coord(z[i], zmin, iwz, nz);
        atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    // exclusive scan of cnt: each thread owns a contiguous run of cells
    const int per = (cells + TPC_BLOCK - 1) / TPC_BLOCK;
    const int c0 = tid * per;
    int c1 = c0 + per;
    if (c1 > cells) c1 = cells;
    int local = 0;
    for (int c = c0; c < c1; ++c) local += cnt[c];
    int total;
    int run = block_exclusive_scan(local, scan_sh, &total);
    for (int c = c0; c < c1; ++c) {
        int v = cnt[c];
        cnt[c] = a + run;             // becomes the scatter cursor
        cstart[base + c] = a + run;
        run += v;
    }
    if (tid == 0) {
        cstart[base + cells] = b;
        SegGrid g = {ymin, zmin, iwy, iwz, ny, nz, 0, 0};
        grid[seg] = g;
    }
    __syncthreads();
    for (int i = a + tid; i < b; i += TPC_BLOCK) {
        float yv = y[i], zv = z[i];
        int c = cell_coord(yv, ymin, iwy, ny) * nz + cell_coord(zv, zmin, iwz, nz);
        int slot = atomicAdd(&cnt[c], 1);
        sy[slot] = yv;
        sz[slot] = zv;
        sid[slot] = i;
    }
}

struct Best {
    float q;
    int32_t u, d;
};

__device__ inline bool better(float q, int32_t u, int32_t d, const Best &b) {
    if (b.u < 0) return true;
    if (q < b.q) return true;
    if (q > b.q) return false;
    if (u != b.u) return u < b.u;
    return d < b.d;
}

// Best triplet of every cluster of segment `seg` (no barriers).
__device__ inline void nb_query_seg(int seg, const int32_t *__restrict__ off, int32_t n_rows,
                                    float win_y, float win_z, float cut_y, float cut_z,
                                    const SegGrid *__restrict__ grid, const int32_t *__restrict__ cstart,
                                    const float *__restrict__ sy, const float *__restrict__ sz,
                                    const int32_t *__restrict__ sid, int32_t *__restrict__ up,
                                    int32_t *__restrict__ dn) {
#pragma clang fp contract(off)
    const int r = seg % n_rows;
    const int a = off[seg], b = off[seg + 1];
    if (r == 0 || r == n_rows - 1) {
        for (int i = a + threadIdx.x; i < b; i += TPC_BLOCK) { up[i] = -1; dn[i] = -1; }
        return;
    }
    const SegGrid gu = grid[seg + 1], gd = grid[seg - 1];
    const int baseu = off[seg + 1] + seg + 1, based = off[seg - 1] + seg - 1;
    for (int j = a + threadIdx.x; j < b; j += TPC_BLOCK) {
        const float yh = sy[j], zh = sz[j];
        const int32_t h = sid[j];
        Best best = {0.f, -1, -1};
        if (gu.ny > 0 && gd.ny > 0) {
            const int cyu = cell_coord(yh, gu.y0, gu.iwy, gu.ny), czu = cell_coord(zh, gu.z0, gu.iwz, gu.nz);
            const int cyd = cell_coord(yh, gd.y0, gd.iwy, gd.ny), czd = cell_coord(zh, gd.z0, gd.iwz, gd.nz);
            const int zu0 = czu > 0 ? czu - 1 : 0, zu1 = czu < gu.nz - 1 ? czu + 1 : gu.nz - 1;
            const int zd0 = czd > 0 ? czd - 1 : 0, zd1 = czd < gd.nz - 1 ? czd + 1 : gd.nz - 1;
            const int yu0 = cyu > 0 ? cyu - 1 : 0, yu1 = cyu < gu.ny - 1 ? cyu + 1 : gu.ny - 1;
            const int yd0 = cyd > 0 ? cyd - 1 : 0, yd1 = cyd < gd.ny - 1 ? cyd + 1 : gd.ny - 1;
            for (int iyu = yu0; iyu <= yu1; ++iyu) {
                const int ue0 = cstart[baseu + iyu * gu.nz + zu0];
                const int ue1 = cstart[baseu + iyu * gu.nz + zu1 + 1];
                for (int ku = ue0; ku < ue1; ++ku) {
                    const float ay = sy[ku] - yh;
                    const float az = sz[ku] - zh;
                    if (!(fabsf(ay) <= win_y && fabsf(az) <= win_z)) continue;
                    const int32_t u = sid[ku];
                    for (int iyd = yd0; iyd <= yd1; ++iyd) {
                        const int de0 = cstart[based + iyd * gd.nz + zd0];
                        const int de1 = cstart[based + iyd * gd.nz + zd1 + 1];
                        for (int kd = de0; kd < de1; ++kd) {
                            const float by = yh - sy[kd];
                            const float bz = zh - sz[kd];
                            if (!(fabsf(by) <= win_y && fabsf(bz) <= win_z)) continue;
                            const float dy = ay - by;
                            const float dz = az - bz;
                            if (!(fabsf(dy) <= cut_y && fabsf(dz) <= cut_z)) continue;
                            const float qy = dy * dy;
                            const float qz = dz * dz;
                            const float q = qy + qz;
                            const int32_t d = sid[kd];
                            if (better(q, u, d, best)) { best.q = q; best.u = u; best.d = d; }
                        }
                    }
                }
            }
        }
        up[h] = best.u;
        dn[h] = best.d;
    }
}

}  // namespace tpc_nb
