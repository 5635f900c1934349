// Internal declarations shared by the kernels and the C-ABI of libtpcreco.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpcreco.h"

#define TPC_MAX_ROWS 256
#define TPC_BLOCK 256          // threads per workgroup: four 64-wide wavefronts
#define TPC_WAVE 64
#define TPC_CELL_CAP 4096      // neighbour-search cells per pad row (LDS histogram size)
#define TPC_SPARSE_GRID 2048   // grid of the kernels that act on few segments (grid-stride; a multiple of 8) ...
#define TPC_SPARSE_ROW 256     // ... when rows hold fewer clusters than this on average

struct GraphCache;
struct tpc_context {
    tpc_config cfg;            // row_x points at row_x_host below
    float row_x_host[TPC_MAX_ROWS];
    float *d_row_x;            // device copy of the row table
    int device;
    int persist_grid;          // resident workgroups of the persistent kernel
    GraphCache *graphs;        // instantiated graphs of TPC_MODE_PERSISTENT_GRAPH
};

// Per-segment neighbour-search grid: cell (iy, iz) of a cluster is
// clamp(floor((y - y0) * iwy)), clamp(floor((z - z0) * iwz)); cell id iy*nz+iz.
struct SegGrid {
    float y0, z0, iwy, iwz;
    int32_t ny, nz, pad0, pad1;
};

// Workspace carving: every buffer starts on a 256-byte boundary.  With a
// null base only the size is computed (no pointer is formed).
struct WsCarver {
    char *base;
    size_t off;
    __host__ __device__ explicit WsCarver(void *b) : base(static_cast<char *>(b)), off(0) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct NbWs {
    SegGrid *grid;      // [NR]
    int32_t *cstart;    // [N + NR + 1]: cell starts of segment s at row_offsets[s] + s
    float *sy, *sz;     // [N] clusters sorted by cell within each segment
    int32_t *sid;       // [N] their global ids
    int32_t *order;     // [TPC_NB_PARTS NR] parts of dense h-rows largest first, then the rest
};

struct CaWs {
    unsigned long long *claim;   // [N] smallest claim key per cluster
    unsigned long long *pack;    // [N] (distance << 32) | lowest chain member in the row block
    int32_t *dlk;                // [N] kept link down, -1 if none
    int2 *cc;                    // [N] at a bottom: (chain length, hit offset of the chain core or
                                 // -1 if no seed), read together; (0, -1) elsewhere
    int32_t *cend;               // [N] at a bottom: the up link of its chain's top (top end candidate)
    int2 *mrec;                  // [N] at a block-local lowest member that is not its chain's
                                 // bottom: (chain bottom, position from it)
    int32_t *fbot;               // [N] at a seed's first cluster: the chain bottom, else -1
    int32_t *flen;               // [N] at a seed's first cluster: seed length
    int32_t *segcnt, *seghits;   // [NR] seeds / seed hits starting in the segment
    int32_t *segbs, *segbh;      // [NR] exclusive prefixes of the above
    int32_t *chunk_c, *chunk_h;  // [ceil(NR / TPC_SCAN_CHUNK)] chunk sums, then their prefixes
};

#define TPC_SCAN_CHUNK 1024      // segments per chunk of the two-level segment scan
#define TPC_SCAN_DIRECT 16384    // up to this many segments one workgroup scans them directly

size_t nb_ws_layout(void *ws, int64_t N, int64_t NR, NbWs *out);
size_t ca_ws_layout(void *ws, int64_t N, int64_t NR, CaWs *out);
size_t chi2_ws_layout(void *ws, int64_t cap_seeds, double **part);
// Length order of the seeds for the fit: order[cap_seeds], the per-length
// bin starts and cursors, the number of ordered seeds.  Fits of at least
// TPC_FIT_ORDER_MIN seed slots run in that order.
struct FitOrderWs {
    int32_t *order, *hist, *cur, *n;
};
#define TPC_FIT_ORDER_MIN 4096
size_t fit_ws_layout(void *ws, int64_t cap_seeds, int64_t cap_hits, double **part, float2 **hyz,
                     FitOrderWs *ord = nullptr);
hipError_t launch_gather(const tpc_frames *fr, const tpc_seeds *sd, float2 *hyz, hipStream_t st);
size_t adj_ws_layout(void *ws, int64_t cap_hits, int64_t cap_seeds, int64_t n_fs, int32_t n_rows,
                     int32_t K, float2 **g, double **tape, float2 **partial, float2 **hyz);

struct PersistArgs;
size_t persist_ws_layout(void *ws, int64_t N, int64_t NR, int64_t cap_seeds, int64_t cap_hits,
                         PersistArgs *P);
int persist_grid(const tpc_context *ctx);
hipError_t launch_persistent(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                             const tpc_seeds *sd, const tpc_tracks *tr, int32_t *dev_status,
                             void *ws, int grid, int sort_fit, int fit_block, int fit_spt, hipStream_t st);
hipError_t launch_fit_shaped(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                             const tpc_tracks *tr, void *ws, int block, int spt, hipStream_t st);

size_t follow_ws_layout(void *ws, int64_t N, int64_t NR, void *index_out);

size_t ctf_ws_layout(void *ws, int64_t N, int64_t NR, int64_t cap_seeds, void *out);
hipError_t launch_ctf_build(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                            const int32_t *rows, const tpc_tracks *tr, float qy, float qz,
                            const tpc_ctf_arrays *out, void *ws, hipStream_t st);

#define TPC_RANS_MAX_RANGE (1 << 20)   // widest symbol range max - min + 1 of one array
struct RansWs {
    int32_t *mm;                 // min, max, status, table bytes, histogram offset, window flag, centre
    uint32_t *counts;            // [TPC_RANS_MAX_RANGE] histogram
    uint4 *fc;                   // [TPC_RANS_MAX_RANGE] (frequency, cumulative frequency, reciprocal, shifts)
    uint32_t *wcount, *wstart;   // [nb], [nb + 1] words per coding block, their prefix
    uint32_t *states;            // [nb][64] final coder states
    uint16_t *scratch;           // [nb][B] word stack of each block
};
size_t rans_ws_layout(void *ws, int64_t n, int32_t B, RansWs *out);
struct RansJob {
    const int32_t *sym;
    int64_t n;                 // symbols, or their upper bound when n_dev is given
    const int64_t *n_dev;      // optional device count
    uint8_t *out;
    uint64_t cap;
    uint64_t *out_size;
    int32_t *dev_status;
};
size_t rans_batch_ws_bytes(int count, const RansJob *jobs, int32_t B);
hipError_t launch_rans_batch(int count, const RansJob *jobs, int32_t L, int32_t B, void *ws,
                             hipStream_t st);
hipError_t launch_follow(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                         double gate, int32_t max_miss, int32_t *rows, const tpc_tracks *tr,
                         void *ws, hipStream_t st);

// launchers (return hipError_t of the last launch)
hipError_t launch_neighbours(const tpc_context *ctx, const tpc_frames *fr, int32_t *up,
                             int32_t *dn, const NbWs &ws, hipStream_t st);
hipError_t launch_ca_seed(const tpc_context *ctx, const tpc_frames *fr, const int32_t *up,
                          const int32_t *dn, const tpc_seeds *sd, int32_t *dev_status,
                          const CaWs &ws, hipStream_t st);
hipError_t launch_fit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                      const float *map, const tpc_tracks *tr, double *ckpt, void *ws, hipStream_t st);
hipError_t launch_chi2_sum(const tpc_seeds *sd, const tpc_tracks *tr, float *loss, void *ws,
                           hipStream_t st);
hipError_t launch_adjoint(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                          const float *map, const tpc_tracks *tr, const double *ckpt,
                          const float *dloss, float *grad_map, void *ws, hipStream_t st);

// ---------------------------------------------------------------------------
// device helpers

// Workgroups go to the eight XCDs round-robin by block id, and each XCD has
// its own L2.  Segment kernels renumber their blocks so that every XCD takes
// one contiguous range of segments: the rows r-1, r, r+1 that a segment's
// work touches are then mostly read through the same L2.  A bijection on
// [0, G).
#define TPC_XCDS 8
__device__ inline int xcd_item(int b, int G) {
    const int x = b % TPC_XCDS, j = b / TPC_XCDS;
    const int q = G / TPC_XCDS, r = G % TPC_XCDS;
    return x * q + (x < r ? x : r) + j;
}

__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & (TPC_WAVE - 1);
#pragma unroll
    for (int d = 1; d < TPC_WAVE; d <<= 1) {
        int t = __shfl_up(v, d, TPC_WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// Seed-length bins hist[0 .. TPC_MAX_ROWS] -> their starts in descending
// length order, and the number of seeds into *total (one whole wavefront:
// lane l takes the bins TPC_MAX_ROWS - 5l down to TPC_MAX_ROWS - 5l - 4,
// then a wave scan of the lanes' sums).
__device__ inline void len_starts_wave(int32_t *hist, int32_t *total) {
    static_assert(5 * TPC_WAVE > TPC_MAX_ROWS, "five bins per lane cover every length");
    const int l = threadIdx.x & (TPC_WAVE - 1);
    int c[5], sum = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int len = TPC_MAX_ROWS - 5 * l - q;
        c[q] = len >= 0 ? hist[len] : 0;
        sum += c[q];
    }
    const int inc = wave_inclusive_scan(sum);
    int run = inc - sum;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int len = TPC_MAX_ROWS - 5 * l - q;
        if (len >= 0) hist[len] = run;
        run += c[q];
    }
    if (l == TPC_WAVE - 1) *total = inc;
}

// Exclusive scan over the TPC_BLOCK threads of a workgroup; returns the prefix
// of this thread and writes the block total to *total.  `sh` holds
// TPC_BLOCK / TPC_WAVE ints of LDS.  Contains barriers: call from every thread.
__device__ inline int block_exclusive_scan(int v, int *sh, int *total) {
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int wid = threadIdx.x / TPC_WAVE;
    int inc = wave_inclusive_scan(v);
    if (lane == TPC_WAVE - 1) sh[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < TPC_BLOCK / TPC_WAVE; ++w) {
        int s = sh[w];
        before += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// A permutation of [0, n) into order: items by descending key(i) in
// [0, TPC_ORDER_BINS], any order within a key (one workgroup of TPC_BLOCK
// threads, a counting sort; contains barriers).  start: TPC_ORDER_BINS + 1
// ints of LDS, sh: TPC_BLOCK / TPC_WAVE ints of LDS.
#define TPC_ORDER_BINS 512
template <class Key>
__device__ inline void order_desc(int n, Key key, int32_t *order, int *start, int *sh) {
    static_assert(3 * TPC_BLOCK > TPC_ORDER_BINS, "three bins per thread cover every key");
    const int tid = threadIdx.x;
    for (int k = tid; k <= TPC_ORDER_BINS; k += TPC_BLOCK) start[k] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += TPC_BLOCK) atomicAdd(&start[key(i)], 1);
    __syncthreads();
    // thread t takes keys TPC_ORDER_BINS - 3t down to TPC_ORDER_BINS - 3t - 2
    int c[3], sum = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int k = TPC_ORDER_BINS - 3 * tid - q;
        c[q] = k >= 0 ? start[k] : 0;
        sum += c[q];
    }
    int total;
    int run = block_exclusive_scan(sum, sh, &total);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int k = TPC_ORDER_BINS - 3 * tid - q;
        if (k >= 0) start[k] = run;
        run += c[q];
    }
    __syncthreads();
    for (int i = tid; i < n; i += TPC_BLOCK) order[atomicAdd(&start[key(i)], 1)] = i;
}

// Size key of segment s for order_desc: 1 + its clusters / 128 (capped),
// 0 if empty.
__device__ inline int seg_size_key(const int32_t *off, int s) {
    const int b = (off[s + 1] - off[s]) >> 7;
    return off[s + 1] == off[s] ? 0 : 1 + (b < TPC_ORDER_BINS - 1 ? b : TPC_ORDER_BINS - 1);
}

__device__ inline float wave_min(float v) {
#pragma unroll
    for (int d = TPC_WAVE / 2; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, TPC_WAVE));
    return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
    for (int d = TPC_WAVE / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, TPC_WAVE));
    return v;
}
