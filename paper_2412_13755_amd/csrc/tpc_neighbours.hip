// Neighbour search stage kernels: one workgroup per (frame, sector, row)
// segment; the per-segment work is in tpc_nb_device.hpp.  nb_bin only works
// on dense rows and their neighbouring rows (z-sorted copies), and
// nb_query_dense only on dense rows.
#include "tpc_nb_device.hpp"

// Dense h-rows of frames of dense rows are searched in TPC_NB_PARTS parts
// of about equal size, each by its own workgroup (two measured faster than
// whole rows, three or four parts).
#ifndef TPC_NB_PARTS
#define TPC_NB_PARTS 2
#endif

namespace {

__global__ void __launch_bounds__(TPC_BLOCK)
nb_bin(const int32_t *__restrict__ off, int32_t NR, int32_t n_rows, const float *__restrict__ y,
       const float *__restrict__ z, float win_y, float win_z, SegGrid *grid, int32_t *cstart, float *sy,
       float *sz, int32_t *sid) {
    __shared__ tpc_nb::BinLdsPerm L;
    // xcd_item keeps each workgroup in its XCD's contiguous range of
    // segments (the grid is NR or a multiple of 8); taking the largest rows
    // first, as the dense query does, made the binning slower
    for (int it = blockIdx.x; it < NR; it += gridDim.x)
        tpc_nb::nb_bin_seg(xcd_item(it, NR), n_rows, off, y, z, win_y, win_z, grid, cstart, sy, sz, sid, L);
}

// Rows whose neighbour rows fit the small LDS form (18 KB per workgroup).
__global__ void __launch_bounds__(TPC_BLOCK)
nb_query_small(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
               const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z,
               int32_t *up, int32_t *dn) {
    __shared__ tpc_nb::PairLdsSmall L;
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    tpc_nb::nb_query_seg(seg, off, n_rows, y, z, win_y, win_z, cut_y, cut_z, nullptr, nullptr, nullptr,
                         nullptr, nullptr, up, dn, L, tpc_nb::NB_SMALL);
}

// Rows whose neighbour rows fit the large LDS form.
__global__ void __launch_bounds__(TPC_BLOCK)
nb_query(const int32_t *__restrict__ off, int32_t n_rows, const float *__restrict__ y,
         const float *__restrict__ z, float win_y, float win_z, float cut_y, float cut_z,
         const SegGrid *grid, const int32_t *cstart, const float *sy, const float *sz,
         const int32_t *sid, int32_t *up, int32_t *dn) {
    __shared__ tpc_nb::PairLds L;
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    tpc_nb::nb_query_seg(seg, off, n_rows, y, z, win_y, win_z, cut_y, cut_z, grid, cstart, sy,
                         sz, sid, up, dn, L, tpc_nb::NB_LARGE);
}

// The order in which the dense query takes its work items, item
// TPC_NB_PARTS s + q being part q of dense h-row s: by descending size in
// steps of 128 clusters (the largest start first, so the last workgroups to
// finish are small ones), then the items with nothing to do.
__global__ void __launch_bounds__(TPC_BLOCK)
nb_dense_order(const int32_t *__restrict__ off, int32_t NR, int32_t n_rows, int32_t *__restrict__ order) {
    __shared__ int start[TPC_ORDER_BINS + 1];
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    order_desc(TPC_NB_PARTS * NR, [&](int i) {
        const int s = i / TPC_NB_PARTS, q = i % TPC_NB_PARTS;
        if (!tpc_nb::dense_hrow(off, s, n_rows)) return 0;
        const int n = tpc_nb::seg_size(off, s);
        const int ps = tpc_nb::dense_split(n, q + 1, TPC_NB_PARTS) - tpc_nb::dense_split(n, q, TPC_NB_PARTS);
        const int b = ps >> 7;
        return ps == 0 ? 0 : 1 + (b < TPC_ORDER_BINS - 1 ? b : TPC_ORDER_BINS - 1);
    }, order, start, sh);
}

// Dense rows: slabs of the z-sorted rows, searched in LDS.  Four wavefronts
// per SIMD (the LDS allows four workgroups per CU): at most 128 VGPRs.
// order: the work items of nb_dense_order (row parts, largest first), or
// null for whole rows in the XCD ranges of xcd_item.
__global__ void __launch_bounds__(TPC_BLOCK, 4)
nb_query_dense(const int32_t *__restrict__ off, int32_t NR, int32_t n_rows, float win_y, float win_z, float cut_y,
               float cut_z, const SegGrid *grid, const int32_t *cstart, const float *sy, const float *sz,
               const int32_t *sid, const int32_t *__restrict__ order, int32_t *up, int32_t *dn) {
    __shared__ tpc_nb::DenseLds L;
    // one call site of the search for both forms: a second inlined copy
    // took the kernel past its 128 VGPRs into scratch spills
    const int items = order ? TPC_NB_PARTS * NR : NR;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        int seg, part = 0, parts = 1;
        if (order) {
            const int item = order[it];
            seg = item / TPC_NB_PARTS;
            part = item % TPC_NB_PARTS;
            parts = TPC_NB_PARTS;
        } else {
            seg = xcd_item(it, NR);
        }
        tpc_nb::nb_dense_seg(seg, off, n_rows, win_y, win_z, cut_y, cut_z, grid, cstart, sy, sz, sid, up, dn, L,
                             part, parts);
    }
}

}  // namespace


hipError_t launch_neighbours(const tpc_context *ctx, const tpc_frames *fr, int32_t *up,
                             int32_t *dn, const NbWs &ws, hipStream_t st) {
    const int NR = fr->n_frames * ctx->cfg.n_sectors * ctx->cfg.n_rows;
    const tpc_config &c = ctx->cfg;
    // the binning and the dense query only work on dense rows and their
    // neighbours: on frames whose rows are small on average a grid of at
    // most TPC_SPARSE_GRID workgroups strides over the segments (no
    // per-segment dispatch for segments with nothing to do); otherwise one
    // workgroup per segment, so heavy segments run side by side
    const bool sparse = (int64_t)fr->n_clusters < (int64_t)TPC_SPARSE_ROW * NR;
    const int gs = sparse && NR > TPC_SPARSE_GRID ? TPC_SPARSE_GRID : NR;
    // frames of dense rows: the dense query takes parts of the dense h-rows,
    // the largest first, so that the tail of a grid of workgroups of very
    // different lengths is made of short ones
    const int32_t *order = nullptr;
    if (!sparse) {
        hipLaunchKernelGGL(nb_dense_order, dim3(1), dim3(TPC_BLOCK), 0, st, fr->row_offsets, NR, c.n_rows,
                           ws.order);
        order = ws.order;
    }
    hipLaunchKernelGGL(nb_bin, dim3(gs), dim3(TPC_BLOCK), 0, st, fr->row_offsets, NR, c.n_rows, fr->y,
                       fr->z, c.win_y, c.win_z, ws.grid, ws.cstart, ws.sy, ws.sz, ws.sid);
    hipLaunchKernelGGL(nb_query_small, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows,
                       fr->y, fr->z, c.win_y, c.win_z, c.cut_y, c.cut_z, up, dn);
    hipLaunchKernelGGL(nb_query, dim3(NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, c.n_rows, fr->y,
                       fr->z, c.win_y, c.win_z, c.cut_y, c.cut_z, ws.grid, ws.cstart, ws.sy, ws.sz,
                       ws.sid, up, dn);
    const int gq = order ? TPC_NB_PARTS * NR : gs;
    hipLaunchKernelGGL(nb_query_dense, dim3(gq), dim3(TPC_BLOCK), 0, st, fr->row_offsets, NR, c.n_rows, c.win_y,
                       c.win_z, c.cut_y, c.cut_z, ws.grid, ws.cstart, ws.sy, ws.sz, ws.sid, order, up, dn);
    return hipGetLastError();
}

size_t nb_ws_layout(void *ws, int64_t N, int64_t NR, NbWs *out) {
    WsCarver w(ws);
    NbWs l;
    l.grid = w.take<SegGrid>(NR);
    l.cstart = w.take<int32_t>(N + NR + 1);
    l.sy = w.take<float>(N);
    l.sz = w.take<float>(N);
    l.sid = w.take<int32_t>(N);
    l.order = w.take<int32_t>(TPC_NB_PARTS * NR);
    if (out) *out = l;
    return (w.off + 255) & ~size_t(255);
}
