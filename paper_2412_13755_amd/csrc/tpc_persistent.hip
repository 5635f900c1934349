// Persistent form of the path (gfx950): neighbour search and seeding of all
// frames in one launch of a grid sized to what the device holds at once
// (occupancy x compute units), then the fit as one following launch.  Every
// phase runs the same per-segment device functions as the stage kernels,
// looping over its work items grid-stride, so results are identical to the
// stage path.  Phases are separated by a grid-wide barrier: an arrival
// counter and a generation word in device memory, with agent-scope fences
// on both sides (the eight XCDs keep separate L2 caches).  A waiting
// workgroup polls with a sleep and gives up after a bounded number of polls,
// setting an error flag that makes every workgroup leave, so the kernel
// always terminates.  The phases share one LDS union.
//
// Phases:  bin | query | links + block ranking | tops + claims | firsts |
//          chunk sums | chunk scan (one workgroup) | segment scan |
//          place + length histogram | members + length scan (one workgroup) |
//          gather hit coordinates + order by length
// (firsts and place take a segment per wavefront; before the binning, every thread flags segments: those needing a z-sorted
// copy and the dense h-rows go to two work lists, so that those phases hand
// out only segments with work; tops and members, whose work is per cluster,
// stride over the clusters instead of the segments)
// The fit is not a phase: its ~230 registers per lane would cap the
// occupancy of every phase at two wavefronts per SIMD.  It runs next, over
// the seeds longest first (with sort_fit), so the lanes of a wavefront carry
// seeds of similar length (the loop length is the seed length).
#include "tpc_ca_device.hpp"
#include "tpc_fit_common.hpp"
#include "tpc_nb_device.hpp"

#define TPC_SPIN_LIMIT (1 << 22)   // polls before a barrier wait is abandoned
#define TPC_BAR_GROUPS 8           // arrival groups of the grid barrier
#define TPC_BAR_STRIDE 16          // words between barrier counters (64 bytes)
#define TPC_BAR_WORDS (TPC_BAR_STRIDE * (TPC_BAR_GROUPS + 1))

struct PersistArgs {
    // frames
    const int32_t *off;
    const float *y, *z;
    int32_t N, NR, NB, n_rows, n_sectors;   // NB: chain-ranking blocks
    float win_y, win_z, cut_y, cut_z;
    int32_t min_hits;
    // outputs
    int32_t *up, *dn;
    tpc_seeds sd;
    int32_t *dev_status;
    FitArgs F;
    // workspace
    NbWs nb;
    CaWs ca;
    unsigned *bar;       // [TPC_BAR_WORDS] top count, top generation, then per group
                         // (every TPC_BAR_STRIDE words) count, generation
    int32_t *err;        // [1]
    int32_t *chunk_c, *chunk_h;   // [nchunks]
    int32_t *len_hist;   // [TPC_MAX_ROWS + 1], then bin starts
    int32_t *len_cur;    // [TPC_MAX_ROWS + 1]
    int32_t *perm;       // [cap_seeds]
    int32_t *n_placed;   // [1]
    int32_t *bin_list, *dense_list;   // [NR] segments needing a z-sorted copy / dense h-rows
    int32_t *n_lists;    // [2] their lengths
    float2 *hyz;         // [cap_hits] seed-ordered hit coordinates
    int32_t nchunks;
    int32_t sort_fit;
};

namespace {

// Wait (thread 0 of a workgroup) until *w differs from `seen`; false if the
// bounded polling runs out (then sets the error flag) or another workgroup
// has set it.
__device__ inline bool wait_change(const PersistArgs &P, unsigned *w, unsigned seen) {
    int spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == seen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > TPC_SPIN_LIMIT) {
            atomicExch(P.err, 1);
            return false;
        }
        if (__hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    }
    return true;
}

// Grid barrier in two levels, so that no single word takes every arrival or
// every poll: workgroups arrive at one of up to TPC_BAR_GROUPS group
// counters (block id mod groups); the last arrival of each group arrives at
// the top counter, the last of those advances the top generation, and each
// group's last arrival then advances its group's generation, which the rest
// of the group polls.  Counters are reset by their last arrival before the
// release, so a workgroup can never see the next barrier's count early.
__device__ inline bool grid_sync(const PersistArgs &P) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int good = 1;
        __threadfence();
        const int G = gridDim.x, ng = G < TPC_BAR_GROUPS ? G : TPC_BAR_GROUPS;
        const int g = blockIdx.x % ng, members = (G - g + ng - 1) / ng;
        unsigned *gc = P.bar + TPC_BAR_STRIDE * (g + 1), *gg = gc + 1;
        const unsigned ggen = __hip_atomic_load(gg, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(gc, 1u);
        if (arrived == (unsigned)members - 1) {
            __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned gen = __hip_atomic_load(&P.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned top = atomicAdd(&P.bar[0], 1u);
            if (top == (unsigned)ng - 1) {
                __hip_atomic_store(&P.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&P.bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else if (!wait_change(P, &P.bar[1], gen)) {
                good = 0;
            }
            __hip_atomic_fetch_add(gg, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else if (!wait_change(P, gg, ggen)) {
            good = 0;
        }
        __threadfence();
        if (__hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) good = 0;
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

__device__ inline int block_sum(int v, int *sh) {
    int tot;
    block_exclusive_scan(v, sh, &tot);
    return tot;
}

__global__ void __launch_bounds__(TPC_BLOCK)
persist_init(PersistArgs P) {
    const int t = blockIdx.x * TPC_BLOCK + threadIdx.x;
    if (t < TPC_BAR_WORDS) P.bar[t] = 0;
    if (t == 0) { *P.err = 0; *P.n_placed = 0; P.n_lists[0] = 0; P.n_lists[1] = 0; }
    if (t <= TPC_MAX_ROWS) { P.len_hist[t] = 0; P.len_cur[t] = 0; }
}

// Four workgroups per CU (the LDS union allows four): at most 128 VGPRs.
__global__ void __launch_bounds__(TPC_BLOCK, 4)
persist_reco(PersistArgs P) {
    __shared__ union {
        tpc_nb::PairLds nb;
        tpc_nb::DenseLds dense;
        tpc_nb::BinLds bin;
        uint32_t caw[TPC_CA_CAP];
        struct {
            int hist[TPC_MAX_ROWS + 1], base[TPC_MAX_ROWS + 1];
        } len;                           // seed lengths (placement and fit order)
    } U;
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    __shared__ int bc[2];
    int *lhist = U.len.hist, *lbase = U.len.base;
    const int G = gridDim.x, bid = blockIdx.x, tid = threadIdx.x;

    // work lists of the binning and the dense query (order within a list is
    // irrelevant: every listed segment is processed whole by one workgroup)
    for (int s = bid * TPC_BLOCK + tid; s < P.NR; s += G * TPC_BLOCK) {
        if (tpc_nb::nb_bin_needed(P.off, s, P.n_rows)) P.bin_list[atomicAdd(&P.n_lists[0], 1)] = s;
        if (tpc_nb::dense_hrow(P.off, s, P.n_rows)) P.dense_list[atomicAdd(&P.n_lists[1], 1)] = s;
    }
    if (!grid_sync(P)) return;
    {
        const int nl = P.n_lists[0];
        for (int k = bid; k < nl; k += G)
            tpc_nb::nb_bin_seg(P.bin_list[k], P.n_rows, P.off, P.y, P.z, P.win_y, P.win_z, P.nb.grid,
                               P.nb.cstart, P.nb.sy, P.nb.sz, P.nb.sid, U.bin);
    }
    if (!grid_sync(P)) return;
    for (int seg = bid; seg < P.NR; seg += G)
        tpc_nb::nb_query_seg(seg, P.off, P.n_rows, P.y, P.z, P.win_y, P.win_z, P.cut_y, P.cut_z,
                             P.nb.grid, P.nb.cstart, P.nb.sy, P.nb.sz, P.nb.sid, P.up, P.dn, U.nb,
                             tpc_nb::NB_NOT_DENSE);
    {
        const int nl = P.n_lists[1];
        for (int k = bid; k < nl; k += G)
            tpc_nb::nb_dense_seg(P.dense_list[k], P.off, P.n_rows, P.win_y, P.win_z, P.cut_y, P.cut_z,
                                 P.nb.grid, P.nb.cstart, P.nb.sy, P.nb.sz, P.nb.sid, P.up, P.dn, U.dense);
    }
    if (!grid_sync(P)) return;
    for (int item = bid; item < P.NB; item += G)
        tpc_ca::ca_block_item(item, P.N, P.n_rows, P.off, P.up, P.dn, P.ca, U.caw);
    if (!grid_sync(P)) return;
    for (int h = bid * TPC_BLOCK + tid; h < P.N; h += G * TPC_BLOCK)
        tpc_ca::ca_tops_one(h, P.N, P.up, P.dn, P.min_hits, P.n_rows, P.ca);
    for (int s = bid * TPC_BLOCK + tid; s < P.NR; s += G * TPC_BLOCK) {   // counted into by the next phase
        P.ca.segcnt[s] = 0;
        P.ca.seghits[s] = 0;
    }
    if (!grid_sync(P)) return;
    // a segment per wavefront (a workgroup's four wavefronts take four)
    for (int seg = bid * (TPC_BLOCK / TPC_WAVE) + tid / TPC_WAVE; seg < P.NR; seg += G * (TPC_BLOCK / TPC_WAVE))
        tpc_ca::ca_firsts_wave(seg, P.N, P.off, P.up, P.dn, P.min_hits, P.ca);
    if (!grid_sync(P)) return;
    // chunk sums of the per-segment seed and hit counts
    for (int ch = bid; ch < P.nchunks; ch += G) {
        const int s0 = ch * TPC_SCAN_CHUNK;
        int vc = 0, vh = 0;
        for (int s = s0 + tid; s < s0 + TPC_SCAN_CHUNK && s < P.NR; s += TPC_BLOCK) {
            vc += P.ca.segcnt[s];
            vh += P.ca.seghits[s];
        }
        const int tc = block_sum(vc, sh);
        const int th = block_sum(vh, sh);
        if (tid == 0) { P.chunk_c[ch] = tc; P.chunk_h[ch] = th; }
    }
    if (!grid_sync(P)) return;
    // exclusive scan of the chunk sums and the totals (one workgroup)
    if (bid == 0) {
        if (tid == 0) { bc[0] = 0; bc[1] = 0; }
        __syncthreads();
        for (int base = 0; base < P.nchunks; base += TPC_BLOCK) {
            const int ch = base + tid;
            const int vc = ch < P.nchunks ? P.chunk_c[ch] : 0;
            const int vh = ch < P.nchunks ? P.chunk_h[ch] : 0;
            int tc, th;
            const int pc = block_exclusive_scan(vc, sh, &tc);
            const int ph = block_exclusive_scan(vh, sh, &th);
            const int cc = bc[0], chh = bc[1];
            if (ch < P.nchunks) { P.chunk_c[ch] = cc + pc; P.chunk_h[ch] = chh + ph; }
            __syncthreads();
            if (tid == 0) { bc[0] = cc + tc; bc[1] = chh + th; }
            __syncthreads();
        }
        if (tid == 0) {
            const int ns = bc[0], nh = bc[1];
            *P.sd.n_seeds = ns;
            *P.sd.n_hits = nh;
            const bool ok = ns <= P.sd.cap_seeds && nh <= P.sd.cap_hits;
            *P.dev_status = ok ? TPC_OK : TPC_ERR_CAPACITY;
            if (ns <= P.sd.cap_seeds) P.sd.offsets[ns] = ok ? nh : 0;
        }
    }
    if (!grid_sync(P)) return;
    // per-segment exclusive prefixes within each chunk
    for (int ch = bid; ch < P.nchunks; ch += G) {
        const int s0 = ch * TPC_SCAN_CHUNK;
        if (tid == 0) { bc[0] = P.chunk_c[ch]; bc[1] = P.chunk_h[ch]; }
        __syncthreads();
        for (int base = s0; base < s0 + TPC_SCAN_CHUNK && base < P.NR; base += TPC_BLOCK) {
            const int s = base + tid;
            const bool in = s < s0 + TPC_SCAN_CHUNK && s < P.NR;
            const int vc = in ? P.ca.segcnt[s] : 0;
            const int vh = in ? P.ca.seghits[s] : 0;
            int tc, th;
            const int pc = block_exclusive_scan(vc, sh, &tc);
            const int ph = block_exclusive_scan(vh, sh, &th);
            const int cc = bc[0], chh = bc[1];
            if (in) { P.ca.segbs[s] = cc + pc; P.ca.segbh[s] = chh + ph; }
            __syncthreads();
            if (tid == 0) { bc[0] = cc + tc; bc[1] = chh + th; }
            __syncthreads();
        }
    }
    if (!grid_sync(P)) return;
    // the seeds' length histogram is counted per workgroup in LDS and added
    // to the global one bin by bin (one global atomic per seed on a few hot
    // bins serialises)
    for (int i = tid; i <= TPC_MAX_ROWS; i += TPC_BLOCK) lhist[i] = 0;
    __syncthreads();
    for (int seg = bid * (TPC_BLOCK / TPC_WAVE) + tid / TPC_WAVE; seg < P.NR; seg += G * (TPC_BLOCK / TPC_WAVE))
        tpc_ca::ca_place_wave(seg, P.N, P.off, P.up, P.y, P.z, P.n_sectors, P.n_rows, P.sd.cap_seeds,
                              P.sd.cap_hits, P.sd, P.ca, P.sort_fit ? lhist : nullptr);
    __syncthreads();
    if (P.sort_fit)
        for (int i = tid; i <= TPC_MAX_ROWS; i += TPC_BLOCK)
            if (lhist[i]) atomicAdd(&P.len_hist[i], lhist[i]);
    if (!grid_sync(P)) return;
    for (int h = bid * TPC_BLOCK + tid; h < P.N; h += G * TPC_BLOCK)
        tpc_ca::ca_members_one(h, P.N, P.y, P.z, P.sd.cap_hits, P.sd, P.ca);
    if (bid == 0 && P.sort_fit) {
        // bin starts in descending length order (the first wavefront)
        if (tid < TPC_WAVE) len_starts_wave(P.len_hist, P.n_placed);
    }
    if (!grid_sync(P)) return;
    {
        // seed-ordered hit coordinates for the fit (unless the seeds carry
        // them); placed seeds form the
        // prefix [0, n_placed): with sort_fit, order them by length
        int H = *P.sd.n_hits;
        if (H > P.sd.cap_hits) H = P.sd.cap_hits;
        if (P.sd.hit_yz) H = 0;         // placement has written them already
        for (int j = bid * TPC_BLOCK + tid; j < H; j += G * TPC_BLOCK) {
            const int32_t id = P.sd.hits[j];
            P.hyz[j] = (uint32_t)id < (uint32_t)P.N ? make_float2(P.y[id], P.z[id]) : make_float2(0.f, 0.f);
        }
        if (P.sort_fit) {
            // the workgroup counts its seeds per length in LDS, reserves one
            // range per length in the global order, then places them (the
            // order within a length is immaterial)
            const int np = *P.n_placed;
            for (int i = tid; i <= TPC_MAX_ROWS; i += TPC_BLOCK) lhist[i] = 0;
            __syncthreads();
            for (int i = bid * TPC_BLOCK + tid; i < np; i += G * TPC_BLOCK) {
                const int n = P.sd.offsets[i + 1] - P.sd.offsets[i];
                atomicAdd(&lhist[n < TPC_MAX_ROWS ? (n > 0 ? n : 0) : TPC_MAX_ROWS], 1);
            }
            __syncthreads();
            for (int i = tid; i <= TPC_MAX_ROWS; i += TPC_BLOCK) {
                const int c = lhist[i];
                lbase[i] = c ? P.len_hist[i] + atomicAdd(&P.len_cur[i], c) : 0;
                lhist[i] = 0;
            }
            __syncthreads();
            for (int i = bid * TPC_BLOCK + tid; i < np; i += G * TPC_BLOCK) {
                const int n = P.sd.offsets[i + 1] - P.sd.offsets[i];
                const int len = n < TPC_MAX_ROWS ? (n > 0 ? n : 0) : TPC_MAX_ROWS;
                const int slot = lbase[len] + atomicAdd(&lhist[len], 1);
                if (slot < np) P.perm[slot] = i;
            }
        }
    }
}

__global__ void persist_status(PersistArgs P) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *P.err != 0) *P.dev_status = TPC_ERR_HIP;
}

}  // namespace

size_t persist_ws_layout(void *ws, int64_t N, int64_t NR, int64_t cap_seeds, int64_t cap_hits,
                         PersistArgs *P) {
    WsCarver w(ws);
    NbWs nb;
    CaWs ca;
    // the neighbour and seeding buffers live side by side (both are in use
    // in one launch)
    const size_t nbb = nb_ws_layout(ws ? w.base : nullptr, N, NR, &nb);
    w.off = nbb;
    const size_t cab = ca_ws_layout(ws ? w.base + nbb : nullptr, N, NR, &ca);
    w.off = nbb + cab;
    unsigned *bar = w.take<unsigned>(TPC_BAR_WORDS);
    int32_t *err = w.take<int32_t>(1);
    const int64_t nchunks = (NR + TPC_SCAN_CHUNK - 1) / TPC_SCAN_CHUNK;
    int32_t *cc = w.take<int32_t>(nchunks > 0 ? nchunks : 1);
    int32_t *chh = w.take<int32_t>(nchunks > 0 ? nchunks : 1);
    int32_t *hist = w.take<int32_t>(TPC_MAX_ROWS + 1);
    int32_t *cur = w.take<int32_t>(TPC_MAX_ROWS + 1);
    int32_t *perm = w.take<int32_t>(cap_seeds > 0 ? cap_seeds : 1);
    int32_t *np = w.take<int32_t>(1);
    int32_t *bl = w.take<int32_t>(NR > 0 ? NR : 1);
    int32_t *dl = w.take<int32_t>(NR > 0 ? NR : 1);
    int32_t *nl = w.take<int32_t>(2);
    float2 *hyz = w.take<float2>(cap_hits > 0 ? cap_hits : 1);
    if (P) {
        P->hyz = hyz;
        P->nb = nb;
        P->ca = ca;
        P->bar = bar;
        P->err = err;
        P->chunk_c = cc;
        P->chunk_h = chh;
        P->len_hist = hist;
        P->len_cur = cur;
        P->perm = perm;
        P->n_placed = np;
        P->bin_list = bl;
        P->dense_list = dl;
        P->n_lists = nl;
        P->nchunks = (int32_t)nchunks;
    }
    return (w.off + 255) & ~size_t(255);
}

int persist_grid(const tpc_context *ctx) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_reco, TPC_BLOCK, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) cus = prop.multiProcessorCount;
    return per_cu * cus;
}

hipError_t launch_persistent(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                             const tpc_seeds *sd, const tpc_tracks *tr, int32_t *dev_status,
                             void *ws, int grid, int sort_fit, int fit_block, int fit_spt, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    PersistArgs P;
    P.off = fr->row_offsets;
    P.y = fr->y;
    P.z = fr->z;
    P.N = fr->n_clusters;
    P.NR = fr->n_frames * c.n_sectors * c.n_rows;
    P.NB = fr->n_frames * c.n_sectors * tpc_ca::ca_blocks_per_sector(c.n_rows);
    P.n_rows = c.n_rows;
    P.n_sectors = c.n_sectors;
    P.win_y = c.win_y;
    P.win_z = c.win_z;
    P.cut_y = c.cut_y;
    P.cut_z = c.cut_z;
    P.min_hits = c.min_hits;
    P.up = up;
    P.dn = dn;
    P.sd = *sd;
    P.dev_status = dev_status;
    P.F = make_fit_args(ctx, fr, sd, nullptr);
    P.F.out = *tr;
    P.sort_fit = sort_fit;
    persist_ws_layout(ws, fr->n_clusters, P.NR, sd->cap_seeds, sd->cap_hits, &P);
    if (sd->hit_yz) P.hyz = reinterpret_cast<float2 *>(sd->hit_yz);
    P.F.hyz = P.hyz;
    hipLaunchKernelGGL(persist_init, dim3(2), dim3(TPC_BLOCK), 0, st, P);
    hipLaunchKernelGGL(persist_reco, dim3(grid), dim3(TPC_BLOCK), 0, st, P);
    // the fit follows as its own launch, longest seeds first with sort_fit
    FitArgs F = P.F;
    if (sort_fit) {
        F.order = P.perm;
        F.n_order = P.n_placed;
    }
    launch_fit_args(F, st, true, fit_block, fit_spt);
    hipLaunchKernelGGL(persist_status, dim3(1), dim3(64), 0, st, P);
    return hipGetLastError();
}
