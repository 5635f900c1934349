// C-ABI of libtpcreco: argument validation, workspace sizing and launches.
// Every check that can be made on the host is made before anything is
// enqueued; nothing here allocates except tpc_create (the row table).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "tpc_internal.hpp"
#include "tpc_fit_ms.hpp"
#include "tpc_nb_skip.hpp"
#include "tpc_merge.hpp"
#include "tpc_refit.hpp"
#include "tpc_rans_dec.hpp"

namespace {

thread_local char g_err[512];

tpc_status fail(tpc_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

tpc_status hip_fail(hipError_t e, const char *what) {
    return fail(TPC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t n_segments(const tpc_context *ctx, const tpc_frames *fr) {
    return (int64_t)fr->n_frames * ctx->cfg.n_sectors * ctx->cfg.n_rows;
}

tpc_status check_frames(const tpc_context *ctx, const tpc_frames *fr) {
    if (!ctx) return fail(TPC_ERR_ARG, "null context");
    if (!fr) return fail(TPC_ERR_ARG, "null frames");
    if (fr->n_frames < 1) return fail(TPC_ERR_ARG, "n_frames < 1");
    if (fr->n_clusters < 0) return fail(TPC_ERR_ARG, "n_clusters < 0");
    const int64_t NR = n_segments(ctx, fr);
    if (NR + (int64_t)fr->n_clusters + 1 >= ((int64_t)1 << 31))
        return fail(TPC_ERR_ARG, "clusters plus segments must stay below 2^31");
    if (NR > (int64_t)0x7fffffff) return fail(TPC_ERR_ARG, "too many segments");
    if (!fr->row_offsets) return fail(TPC_ERR_ARG, "null row_offsets");
    if (fr->n_clusters > 0 && (!fr->y || !fr->z)) return fail(TPC_ERR_ARG, "null y or z");
    return TPC_OK;
}

tpc_status check_ws(void *ws, size_t have, size_t need) {
    if (need == 0) return TPC_OK;
    if (!ws) return fail(TPC_ERR_WORKSPACE, "workspace is null, %zu bytes needed", need);
    if (((uintptr_t)ws & 255) != 0) return fail(TPC_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (have < need) return fail(TPC_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
    return TPC_OK;
}

// Seeds hold >= min_hits distinct clusters: default capacities never overflow.
int64_t seed_cap_bound(const tpc_context *ctx, int64_t N) { return N / ctx->cfg.min_hits + 1; }

size_t fit_bytes(int64_t cap_seeds, int64_t cap_hits) {
    return fit_ws_layout(nullptr, cap_seeds, cap_hits, nullptr, nullptr);
}

size_t adjoint_bytes(const tpc_context *ctx, const tpc_frames *fr, int64_t cap_hits, int64_t cap_seeds) {
    const int64_t n_fs = (int64_t)fr->n_frames * ctx->cfg.n_sectors;
    return adj_ws_layout(nullptr, cap_hits, cap_seeds, n_fs, ctx->cfg.n_rows, ctx->cfg.ckpt_rows,
                         nullptr, nullptr, nullptr, nullptr);
}

size_t stage_bytes(const tpc_context *ctx, const tpc_frames *fr, int32_t mask) {
    const int64_t N = fr->n_clusters, NR = n_segments(ctx, fr);
    const int64_t cs = seed_cap_bound(ctx, N);
    size_t b = 0;
    if (mask & TPC_STAGE_NEIGHBOURS) b = std::max(b, nb_ws_layout(nullptr, N, NR, nullptr));
    if (mask & TPC_STAGE_SEED) b = std::max(b, ca_ws_layout(nullptr, N, NR, nullptr));
    if (mask & TPC_STAGE_FIT) b = std::max(b, fit_bytes(cs, N > 0 ? N : 1));
    if (mask & TPC_STAGE_ADJOINT) b = std::max(b, adjoint_bytes(ctx, fr, N > 0 ? N : 1, cs));
    if (mask & TPC_STAGE_PERSISTENT)
        b = std::max(b, persist_ws_layout(nullptr, N, NR, cs, N > 0 ? N : 1, nullptr));
    if (mask & TPC_STAGE_FOLLOW) b = std::max(b, follow_ws_layout(nullptr, N, NR, nullptr));
    if (mask & TPC_STAGE_CTF) b = std::max(b, ctf_ws_layout(nullptr, N, NR, cs, nullptr));
    if (mask & TPC_STAGE_SKIP) b = std::max(b, skip_ws_layout(nullptr, N, NR, nullptr));
    if (mask & TPC_STAGE_SMOOTH) b = std::max(b, smooth_ws_layout(nullptr, cs, N > 0 ? N : 1, nullptr));
    return b;
}

size_t ckpt_bytes(const tpc_context *ctx, const tpc_seeds *sd) {
    const int64_t slots = (int64_t)sd->cap_hits / ctx->cfg.ckpt_rows + sd->cap_seeds + 1;
    return (size_t)slots * 20 * sizeof(double);
}

tpc_status check_seeds_for_fit(const tpc_seeds *sd) {
    if (!sd) return fail(TPC_ERR_ARG, "null seeds");
    if (sd->cap_seeds < 0 || sd->cap_hits < 0) return fail(TPC_ERR_ARG, "negative capacity");
    if (!sd->n_seeds || !sd->offsets) return fail(TPC_ERR_ARG, "null seed counters or offsets");
    if (sd->cap_seeds > 0 && (!sd->hits || !sd->sector || !sd->first_row || !sd->frame))
        return fail(TPC_ERR_ARG, "null seed arrays");
    if (((uintptr_t)sd->hit_yz & 7) != 0) return fail(TPC_ERR_ARG, "hit_yz not 8-byte aligned");
    return TPC_OK;
}

tpc_status check_tracks(const tpc_seeds *sd, const tpc_tracks *tr) {
    if (!tr) return fail(TPC_ERR_ARG, "null tracks");
    if (sd->cap_seeds > 0 && (!tr->x || !tr->par || !tr->cov || !tr->chi2 || !tr->ndf || !tr->status))
        return fail(TPC_ERR_ARG, "null track arrays");
    return TPC_OK;
}

// Material parameters, when given (NULL is accepted here).
tpc_status check_material(const tpc_material *mat) {
    if (!mat) return TPC_OK;
    if (!(mat->x0 > 0.f)) return fail(TPC_ERR_ARG, "x0 must be > 0");
    if (!(mat->mass >= 0.f) || !isfinite(mat->mass)) return fail(TPC_ERR_ARG, "mass must be finite and >= 0");
    if (!(mat->chi2_cut > 0.f)) return fail(TPC_ERR_ARG, "chi2_cut must be > 0");
    if (!(mat->rho >= 0.f) || !isfinite(mat->rho)) return fail(TPC_ERR_ARG, "rho must be finite and >= 0");
    if (mat->rho > 0.f && !(mat->mass > 0.f && mat->z_over_a > 0.f && isfinite(mat->z_over_a) &&
                            mat->mean_exc > 0.f && isfinite(mat->mean_exc)))
        return fail(TPC_ERR_ARG, "energy loss needs mass, z_over_a and mean_exc finite and > 0");
    return TPC_OK;
}

}  // namespace

extern "C" {

const char *tpc_status_string(tpc_status s) {
    switch (s) {
        case TPC_OK: return "TPC_OK";
        case TPC_ERR_ARG: return "TPC_ERR_ARG";
        case TPC_ERR_CAPACITY: return "TPC_ERR_CAPACITY";
        case TPC_ERR_HIP: return "TPC_ERR_HIP";
        case TPC_ERR_UNSUPPORTED: return "TPC_ERR_UNSUPPORTED";
        case TPC_ERR_WORKSPACE: return "TPC_ERR_WORKSPACE";
        default: return "TPC_ERR_UNKNOWN";
    }
}

const char *tpc_last_error(void) { return g_err; }

// Seeding scratch of tpc_ca_seed_noalloc: one array per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is taken once per device (in
// tpc_create, with that device current) and only that address is passed to
// kernels.
#define TPC_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[TPC_NOALLOC_SCRATCH_BYTES];
static void *g_scratch_ptr[TPC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static tpc_status scratch_init(int dev) {
    if (dev < 0 || dev >= TPC_MAX_DEVICES) return fail(TPC_ERR_ARG, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return TPC_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(TPC_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = p;
    return TPC_OK;
}

static void *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (dev >= 0 && dev < TPC_MAX_DEVICES) ? g_scratch_ptr[dev] : nullptr;
}

tpc_status tpc_create(const tpc_config *cfg, tpc_context **out) {
    g_err[0] = 0;
    if (!out) return fail(TPC_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (!cfg) return fail(TPC_ERR_ARG, "null config");
    const tpc_config &c = *cfg;
    if (c.n_sectors < 1) return fail(TPC_ERR_ARG, "n_sectors < 1");
    if (c.n_rows < 3 || c.n_rows > TPC_MAX_ROWS) return fail(TPC_ERR_ARG, "n_rows outside 3..%d", TPC_MAX_ROWS);
    if (!c.row_x) return fail(TPC_ERR_ARG, "null row_x");
    for (int r = 0; r < c.n_rows; ++r) {
        if (!isfinite(c.row_x[r])) return fail(TPC_ERR_ARG, "row_x[%d] not finite", r);
        if (r > 0 && !(c.row_x[r] > c.row_x[r - 1])) return fail(TPC_ERR_ARG, "row_x not increasing at %d", r);
    }
    {
        // the neighbour predicate's second difference assumes equally spaced
        // planes: every pitch within TPC_PITCH_TOL of the mean pitch
        const double mean = ((double)c.row_x[c.n_rows - 1] - (double)c.row_x[0]) / (c.n_rows - 1);
        for (int r = 1; r < c.n_rows; ++r) {
            const double p = (double)c.row_x[r] - (double)c.row_x[r - 1];
            if (fabs(p - mean) > TPC_PITCH_TOL * mean)
                return fail(TPC_ERR_ARG, "non-uniform row pitch: row_x[%d] - row_x[%d] = %g, mean %g", r, r - 1, p,
                            mean);
        }
    }
    if (!(fabsf(c.bz) >= 1e-6f) || !isfinite(c.bz)) return fail(TPC_ERR_ARG, "|bz| < 1e-6");
    if (!(c.sigma_y > 0.f) || !(c.sigma_z > 0.f)) return fail(TPC_ERR_ARG, "sigma_y, sigma_z must be > 0");
    if (!(c.win_y > 0.f) || !(c.win_z > 0.f) || !isfinite(c.win_y) || !isfinite(c.win_z))
        return fail(TPC_ERR_ARG, "windows must be finite and > 0");
    if (!(c.cut_y > 0.f) || !(c.cut_z > 0.f)) return fail(TPC_ERR_ARG, "cuts must be > 0");
    if (c.min_hits < 3) return fail(TPC_ERR_ARG, "min_hits < 3");
    if (!(c.max_sin > 0.f && c.max_sin < 1.f)) return fail(TPC_ERR_ARG, "max_sin outside (0, 1)");
    if (!(c.var_sin0 > 0.f) || !(c.var_tgl0 > 0.f) || !(c.var_qpt0 > 0.f))
        return fail(TPC_ERR_ARG, "start variances must be > 0");
    if (c.ckpt_rows < 1 || c.ckpt_rows > 64) return fail(TPC_ERR_ARG, "ckpt_rows outside 1..64");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(TPC_ERR_UNSUPPORTED, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    tpc_context *ctx = new (std::nothrow) tpc_context;
    if (!ctx) return fail(TPC_ERR_ARG, "out of host memory");
    ctx->cfg = c;
    memcpy(ctx->row_x_host, c.row_x, sizeof(float) * c.n_rows);
    ctx->cfg.row_x = ctx->row_x_host;
    ctx->device = dev;
    ctx->d_row_x = nullptr;
    ctx->graphs = nullptr;
    e = hipMalloc(&ctx->d_row_x, sizeof(float) * TPC_MAX_ROWS);
    if (e != hipSuccess) { delete ctx; return hip_fail(e, "hipMalloc(row table)"); }
    e = hipMemcpy(ctx->d_row_x, ctx->row_x_host, sizeof(float) * c.n_rows, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(ctx->d_row_x); delete ctx; return hip_fail(e, "hipMemcpy(row table)"); }
    ctx->persist_grid = persist_grid(ctx);
    tpc_status ss = scratch_init(dev);
    if (ss) { (void)hipFree(ctx->d_row_x); delete ctx; return ss; }
    *out = ctx;
    return TPC_OK;
}

// Graphs of TPC_MODE_PERSISTENT_GRAPH: one per argument set, keyed by the
// bytes of every argument (zero-filled first, so padding compares equal),
// captured on a stream of the context's own and instantiated once.
struct GraphKey {
    tpc_frames fr;
    const int32_t *up, *dn;
    tpc_seeds sd;
    tpc_tracks tr;
    const int32_t *dev_status;
    const void *ws;
    size_t ws_bytes;
    int32_t grid, sort_fit, fit_block, fit_spt;
};
struct GraphCache {
    std::mutex mu;
    hipStream_t capture = nullptr;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> items;
};
static std::mutex g_graph_create_mu;

static void graphs_free(tpc_context *ctx) {
    GraphCache *g = ctx->graphs;
    if (!g) return;
    for (auto &it : g->items) (void)hipGraphExecDestroy(it.second);
    if (g->capture) (void)hipStreamDestroy(g->capture);
    delete g;
    ctx->graphs = nullptr;
}

static tpc_status graph_replay(const tpc_context *cctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                               const tpc_seeds *sd, const tpc_tracks *tr, int32_t *dev_status, void *ws,
                               size_t ws_bytes, int grid, int sort_fit, int fit_block, int fit_spt,
                               hipStream_t st) {
    tpc_context *ctx = const_cast<tpc_context *>(cctx);   // the cache is the context's mutable part
    GraphKey k;
    memset(&k, 0, sizeof k);
    k.fr = *fr;
    k.up = up;
    k.dn = dn;
    k.sd = *sd;
    k.tr = *tr;
    k.dev_status = dev_status;
    k.ws = ws;
    k.ws_bytes = ws_bytes;
    k.grid = grid;
    k.sort_fit = sort_fit;
    k.fit_block = fit_block;
    k.fit_spt = fit_spt;
    {
        std::lock_guard<std::mutex> lk(g_graph_create_mu);
        if (!ctx->graphs) ctx->graphs = new (std::nothrow) GraphCache;
    }
    GraphCache *g = ctx->graphs;
    if (!g) return fail(TPC_ERR_ARG, "out of host memory");
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (auto &it : g->items)
            if (memcmp(&it.first, &k, sizeof k) == 0) { exec = it.second; break; }
        if (!exec) {
            hipError_t e = hipSuccess;
            if (!g->capture) e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
            e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            const hipError_t le = launch_persistent(ctx, fr, up, dn, sd, tr, dev_status, ws, grid, sort_fit,
                                                    fit_block, fit_spt, g->capture);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(g->capture, &graph);
            if (le != hipSuccess || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(le != hipSuccess ? le : e, "persistent kernel capture");
            }
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            g->items.emplace_back(k, exec);
        }
    }
    const hipError_t e = hipGraphLaunch(exec, st);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "hipGraphLaunch");
}

void tpc_destroy(tpc_context *ctx) {
    if (!ctx) return;
    graphs_free(ctx);
    if (ctx->d_row_x) (void)hipFree(ctx->d_row_x);
    delete ctx;
}

tpc_status tpc_workspace_bytes(const tpc_context *ctx, const tpc_frames *fr, int32_t stage_mask,
                               size_t *bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(TPC_ERR_ARG, "null bytes");
    if (!ctx || !fr) return fail(TPC_ERR_ARG, "null context or frames");
    if (fr->n_frames < 1 || fr->n_clusters < 0) return fail(TPC_ERR_ARG, "bad frame sizes");
    if ((stage_mask & ~TPC_STAGE_ALL) != 0) return fail(TPC_ERR_ARG, "unknown stage bits");
    *bytes = stage_bytes(ctx, fr, stage_mask);
    return TPC_OK;
}

tpc_status tpc_neighbours(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                          void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if (fr->n_clusters > 0 && (!up || !dn)) return fail(TPC_ERR_ARG, "null up or dn");
    s = check_ws(ws, ws_bytes, stage_bytes(ctx, fr, TPC_STAGE_NEIGHBOURS));
    if (s) return s;
    if (fr->n_clusters == 0) return TPC_OK;
    NbWs l;
    nb_ws_layout(ws, fr->n_clusters, n_segments(ctx, fr), &l);
    hipError_t e = launch_neighbours(ctx, fr, up, dn, l, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "neighbour kernels");
}

tpc_status tpc_neighbours_skip(const tpc_context *ctx, const tpc_frames *fr, int32_t *up, int32_t *dn,
                               void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if (fr->n_clusters > 0 && (!up || !dn)) return fail(TPC_ERR_ARG, "null up or dn");
    s = check_ws(ws, ws_bytes, stage_bytes(ctx, fr, TPC_STAGE_SKIP));
    if (s) return s;
    if (fr->n_clusters == 0) return TPC_OK;
    SkipWs l;
    skip_ws_layout(ws, fr->n_clusters, n_segments(ctx, fr), &l);
    hipError_t e = launch_neighbours_skip(ctx, fr, up, dn, l, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "neighbour kernels");
}

tpc_status tpc_ca_seed(const tpc_context *ctx, const tpc_frames *fr, const int32_t *up,
                       const int32_t *dn, tpc_seeds *sd, int32_t *dev_status, void *ws,
                       size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if (fr->n_clusters > 0 && (!up || !dn)) return fail(TPC_ERR_ARG, "null up or dn");
    if (!sd || !dev_status) return fail(TPC_ERR_ARG, "null seeds or dev_status");
    if (sd->cap_seeds < 0 || sd->cap_hits < 0) return fail(TPC_ERR_ARG, "negative capacity");
    if (!sd->n_seeds || !sd->n_hits || !sd->offsets) return fail(TPC_ERR_ARG, "null seed counters or offsets");
    if (sd->cap_seeds > 0 && (!sd->frame || !sd->sector || !sd->first_row))
        return fail(TPC_ERR_ARG, "null seed arrays");
    if (sd->cap_hits > 0 && !sd->hits) return fail(TPC_ERR_ARG, "null seed hits");
    if (((uintptr_t)sd->hit_yz & 7) != 0) return fail(TPC_ERR_ARG, "hit_yz not 8-byte aligned");
    s = check_ws(ws, ws_bytes, stage_bytes(ctx, fr, TPC_STAGE_SEED));
    if (s) return s;
    CaWs l;
    ca_ws_layout(ws, fr->n_clusters, n_segments(ctx, fr), &l);
    hipError_t e = launch_ca_seed(ctx, fr, up, dn, sd, dev_status, l, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "seeding kernels");
}

tpc_status tpc_ca_seed_noalloc(const tpc_context *ctx, const tpc_frames *fr, const int32_t *up,
                               const int32_t *dn, tpc_seeds *sd, int32_t *dev_status, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if (fr->n_clusters > 0 && (!up || !dn)) return fail(TPC_ERR_ARG, "null up or dn");
    if (!sd || !dev_status) return fail(TPC_ERR_ARG, "null seeds or dev_status");
    if (sd->cap_seeds < 0 || sd->cap_hits < 0) return fail(TPC_ERR_ARG, "negative capacity");
    if (!sd->n_seeds || !sd->n_hits || !sd->offsets) return fail(TPC_ERR_ARG, "null seed counters or offsets");
    if (sd->cap_seeds > 0 && (!sd->frame || !sd->sector || !sd->first_row))
        return fail(TPC_ERR_ARG, "null seed arrays");
    if (sd->cap_hits > 0 && !sd->hits) return fail(TPC_ERR_ARG, "null seed hits");
    if (((uintptr_t)sd->hit_yz & 7) != 0) return fail(TPC_ERR_ARG, "hit_yz not 8-byte aligned");
    const size_t need = ca_ws_layout(nullptr, fr->n_clusters, n_segments(ctx, fr), nullptr);
    if (need > TPC_NOALLOC_SCRATCH_BYTES)
        return fail(TPC_ERR_WORKSPACE, "frames need %zu bytes of seeding scratch, the built-in scratch holds %zu",
                    need, (size_t)TPC_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != ctx->device) return fail(TPC_ERR_ARG, "current device %d is not the context's device %d", dev, ctx->device);
    void *ws = scratch_ptr(dev);
    if (!ws) return fail(TPC_ERR_HIP, "no scratch address for device %d", dev);
    CaWs l;
    ca_ws_layout(ws, fr->n_clusters, n_segments(ctx, fr), &l);
    e = launch_ca_seed(ctx, fr, up, dn, sd, dev_status, l, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "seeding kernels");
}

tpc_status tpc_ckpt_bytes(const tpc_context *ctx, const tpc_seeds *seeds, size_t *bytes) {
    g_err[0] = 0;
    if (!ctx || !seeds || !bytes) return fail(TPC_ERR_ARG, "null argument");
    if (seeds->cap_seeds < 0 || seeds->cap_hits < 0) return fail(TPC_ERR_ARG, "negative capacity");
    *bytes = ckpt_bytes(ctx, seeds);
    return TPC_OK;
}

tpc_status tpc_kalman_fit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                          const float *map, tpc_tracks *tr, void *ckpt, size_t ckpt_bytes_have,
                          void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (ckpt) {
        if (((uintptr_t)ckpt & 7) != 0) return fail(TPC_ERR_ARG, "checkpoint buffer not 8-byte aligned");
        const size_t need = ckpt_bytes(ctx, sd);
        if (ckpt_bytes_have < need)
            return fail(TPC_ERR_WORKSPACE, "checkpoint buffer has %zu bytes, %zu needed", ckpt_bytes_have, need);
    }
    if ((s = check_ws(ws, ws_bytes, fit_bytes(sd->cap_seeds, sd->cap_hits)))) return s;
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_fit(ctx, fr, sd, map, tr, (double *)ckpt, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "fit kernel");
}

tpc_status tpc_kalman_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                                   const tpc_material *mat, tpc_tracks *tr, uint8_t *rejected, void *ws,
                                   size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (!mat) return fail(TPC_ERR_ARG, "null material");
    if ((s = check_material(mat))) return s;
    if ((s = check_ws(ws, ws_bytes, fit_bytes(sd->cap_seeds, sd->cap_hits)))) return s;
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_fit_material(ctx, fr, sd, mat, tr, rejected, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "fit kernel");
}

tpc_status tpc_kalman_fit_rows(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const float *cluster_err, const tpc_material *mat, tpc_tracks *tr,
                               uint8_t *rejected, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if ((s = check_material(mat))) return s;
    if (((uintptr_t)cluster_err & 7) != 0) return fail(TPC_ERR_ARG, "cluster_err not 8-byte aligned");
    if ((s = check_ws(ws, ws_bytes, fit_bytes(sd->cap_seeds, sd->cap_hits)))) return s;
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_fit_rows(ctx, fr, sd, cluster_err, mat, tr, rejected, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "fit kernel");
}

tpc_status tpc_kalman_smooth(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                             const float *cluster_err, const tpc_material *mat, tpc_tracks *tr,
                             uint8_t *rejected, float *hit_par, float *hit_cov, void *ws, size_t ws_bytes,
                             void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if ((s = check_material(mat))) return s;
    if (((uintptr_t)cluster_err & 7) != 0) return fail(TPC_ERR_ARG, "cluster_err not 8-byte aligned");
    if (sd->cap_hits > 0 && (!rejected || !hit_par || !hit_cov))
        return fail(TPC_ERR_ARG, "null rejected, hit_par or hit_cov");
    if ((s = check_ws(ws, ws_bytes, smooth_ws_layout(nullptr, sd->cap_seeds, sd->cap_hits, nullptr)))) return s;
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_smooth(ctx, fr, sd, cluster_err, mat, tr, rejected, hit_par, hit_cov, ws,
                                 (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "fit and smoother kernels");
}

tpc_status tpc_chi2_sum(const tpc_context *ctx, const tpc_seeds *sd, const tpc_tracks *tr,
                        float *loss, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (!ctx) return fail(TPC_ERR_ARG, "null context");
    tpc_status s = check_seeds_for_fit(sd);
    if (s) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (!loss) return fail(TPC_ERR_ARG, "null loss");
    if ((s = check_ws(ws, ws_bytes, chi2_ws_layout(nullptr, sd->cap_seeds, nullptr)))) return s;
    hipError_t e = launch_chi2_sum(sd, tr, loss, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "chi2 sum kernels");
}

tpc_status tpc_fit_adjoint(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                           const float *map, const tpc_tracks *tr, const void *ckpt,
                           size_t ckpt_bytes_have, const float *dloss, float *grad_map, void *ws,
                           size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (!grad_map) return fail(TPC_ERR_ARG, "null grad_map");
    if (!ckpt) return fail(TPC_ERR_ARG, "null checkpoint buffer");
    if (((uintptr_t)ckpt & 7) != 0) return fail(TPC_ERR_ARG, "checkpoint buffer not 8-byte aligned");
    const size_t need_ck = ckpt_bytes(ctx, sd);
    if (ckpt_bytes_have < need_ck)
        return fail(TPC_ERR_WORKSPACE, "checkpoint buffer has %zu bytes, %zu needed", ckpt_bytes_have, need_ck);
    if ((s = check_ws(ws, ws_bytes, adjoint_bytes(ctx, fr, sd->cap_hits, sd->cap_seeds)))) return s;
    hipError_t e = launch_adjoint(ctx, fr, sd, map, tr, (const double *)ckpt, dloss, grad_map, ws,
                                  (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "adjoint kernels");
}

tpc_status tpc_reconstruct(const tpc_context *ctx, const tpc_frames *fr, int32_t mode,
                           const tpc_tune *tune, int32_t *up, int32_t *dn, tpc_seeds *sd,
                           tpc_tracks *tr, int32_t *dev_status, void *ws, size_t ws_bytes,
                           void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if (mode != TPC_MODE_STAGED && mode != TPC_MODE_PERSISTENT && mode != TPC_MODE_PERSISTENT_GRAPH)
        return fail(TPC_ERR_ARG, "unknown mode %d", mode);
    if (fr->n_clusters > 0 && (!up || !dn)) return fail(TPC_ERR_ARG, "null up or dn");
    if (!dev_status) return fail(TPC_ERR_ARG, "null dev_status");
    if ((s = check_seeds_for_fit(sd))) return s;
    if (!sd->n_hits || (sd->cap_hits > 0 && !sd->hits)) return fail(TPC_ERR_ARG, "null seed hits");
    if ((s = check_tracks(sd, tr))) return s;
    if (tune && (tune->grid < 0 || tune->sort_fit < 0 || tune->sort_fit > 1 ||
                 (tune->fit_block != 0 && tune->fit_block != 64 && tune->fit_block != 128 &&
                  tune->fit_block != 256) ||
                 tune->fit_spt < 0 || tune->fit_spt > 64))
        return fail(TPC_ERR_ARG, "bad tune values");
    hipStream_t st = (hipStream_t)stream;
    const int fit_block = tune ? tune->fit_block : 0, fit_spt = tune ? tune->fit_spt : 0;
    if (mode == TPC_MODE_STAGED) {
        if ((s = check_ws(ws, ws_bytes, stage_bytes(ctx, fr, TPC_STAGE_NEIGHBOURS | TPC_STAGE_SEED | TPC_STAGE_FIT))))
            return s;
        if ((s = tpc_neighbours(ctx, fr, up, dn, ws, ws_bytes, stream))) return s;
        if ((s = tpc_ca_seed(ctx, fr, up, dn, sd, dev_status, ws, ws_bytes, stream))) return s;
        hipError_t e = launch_fit_shaped(ctx, fr, sd, tr, ws, fit_block, fit_spt, st);
        return e == hipSuccess ? TPC_OK : hip_fail(e, "fit kernels");
    }
    const int64_t NR = n_segments(ctx, fr);
    if ((s = check_ws(ws, ws_bytes, persist_ws_layout(nullptr, fr->n_clusters, NR, sd->cap_seeds,
                                                      sd->cap_hits, nullptr))))
        return s;
    int grid = ctx->persist_grid;
    if (tune && tune->grid > 0 && tune->grid < grid) grid = tune->grid;
    const int sort_fit = tune ? tune->sort_fit : 1;
    if (mode == TPC_MODE_PERSISTENT_GRAPH)
        return graph_replay(ctx, fr, up, dn, sd, tr, dev_status, ws, ws_bytes, grid, sort_fit, fit_block, fit_spt, st);
    hipError_t e = launch_persistent(ctx, fr, up, dn, sd, tr, dev_status, ws, grid, sort_fit, fit_block, fit_spt, st);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "persistent kernel");
}

tpc_status tpc_track_follow(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                            const tpc_follow_params *prm, int32_t *rows, tpc_tracks *tr, void *ws,
                            size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (!prm) return fail(TPC_ERR_ARG, "null follow parameters");
    if (!(prm->gate_chi2 >= 0.f) || !isfinite(prm->gate_chi2)) return fail(TPC_ERR_ARG, "gate_chi2 must be finite and >= 0");
    if (prm->max_miss < 0 || prm->max_miss > ctx->cfg.n_rows) return fail(TPC_ERR_ARG, "max_miss outside 0..n_rows");
    if (sd->cap_seeds > 0 && !rows) return fail(TPC_ERR_ARG, "null rows");
    if ((int64_t)sd->cap_seeds * ctx->cfg.n_rows >= ((int64_t)1 << 31))
        return fail(TPC_ERR_ARG, "cap_seeds * n_rows must stay below 2^31");
    if ((s = check_ws(ws, ws_bytes, stage_bytes(ctx, fr, TPC_STAGE_FOLLOW)))) return s;
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_follow(ctx, fr, sd, (double)prm->gate_chi2, prm->max_miss, rows, tr, ws,
                                 (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "follow kernels");
}

tpc_status tpc_track_merge(const tpc_context *ctx, const tpc_seeds *sd, const tpc_tracks *tr, float chi2_cut,
                           int32_t *next, int32_t *prev, float *chi2, float *merged_par, float *merged_cov,
                           int32_t *leg, float *leg_chi2, void *stream) {
    g_err[0] = 0;
    if (!ctx) return fail(TPC_ERR_ARG, "null context");
    tpc_status s = check_seeds_for_fit(sd);
    if (s) return s;
    if ((s = check_tracks(sd, tr))) return s;
    if (!(chi2_cut > 0.f) || !isfinite(chi2_cut)) return fail(TPC_ERR_ARG, "chi2_cut must be finite and > 0");
    if (sd->cap_seeds > 0 && (!next || !prev || !chi2)) return fail(TPC_ERR_ARG, "null merge outputs");
    if (!merged_par != !merged_cov) return fail(TPC_ERR_ARG, "merged_par and merged_cov must both be given or both null");
    if (!leg != !leg_chi2) return fail(TPC_ERR_ARG, "leg and leg_chi2 must both be given or both null");
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_merge(ctx, sd, tr, (double)chi2_cut, next, prev, chi2, merged_par, merged_cov, leg,
                                leg_chi2, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "merge kernels");
}

tpc_status tpc_track_refit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                           const tpc_tracks *seg, const int32_t *next, const int32_t *prev, const int32_t *leg,
                           const float *map, int32_t *track_id, tpc_tracks *out, float *loop_par,
                           float *loop_cov, float *loop_chi2, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if (!seg || (sd->cap_seeds > 0 && !seg->status)) return fail(TPC_ERR_ARG, "null segment status");
    if ((s = check_tracks(sd, out))) return s;
    if (sd->cap_seeds > 0 && (!next || !prev || !track_id)) return fail(TPC_ERR_ARG, "null links or track ids");
    const int nl = (loop_par != nullptr) + (loop_cov != nullptr) + (loop_chi2 != nullptr);
    if (nl != 0 && nl != 3) return fail(TPC_ERR_ARG, "loop_par, loop_cov and loop_chi2 must all be given or all null");
    if (nl && !leg) return fail(TPC_ERR_ARG, "looper circles need leg links");
    if (sd->cap_seeds == 0) return TPC_OK;
    hipError_t e = launch_refit(ctx, fr, sd, seg, next, prev, leg, map, track_id, out, loop_par, loop_cov,
                                loop_chi2, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "refit kernels");
}

tpc_status tpc_ctf_build(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                         const int32_t *rows, const tpc_tracks *tr, float qy, float qz,
                         const tpc_ctf_arrays *out, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_frames(ctx, fr);
    if (s) return s;
    if ((s = check_seeds_for_fit(sd))) return s;
    if (!tr || (sd->cap_seeds > 0 && !tr->status)) return fail(TPC_ERR_ARG, "null track status");
    if (sd->cap_seeds > 0 && !rows) return fail(TPC_ERR_ARG, "null rows");
    if (!(qy > 0.f) || !(qz > 0.f) || !isfinite(qy) || !isfinite(qz))
        return fail(TPC_ERR_ARG, "quantisation steps must be finite and > 0");
    if (!out || !out->counts) return fail(TPC_ERR_ARG, "null output arrays or counts");
    int32_t *const *a = &out->trk_seg;
    for (int k = 0; k < TPC_CTF_ARRAYS; ++k)
        if (!a[k]) return fail(TPC_ERR_ARG, "null output array %d", k);
    const int64_t NR = n_segments(ctx, fr);
    if ((s = check_ws(ws, ws_bytes, ctf_ws_layout(nullptr, fr->n_clusters, NR, sd->cap_seeds, nullptr))))
        return s;
    hipError_t e = launch_ctf_build(ctx, fr, sd, rows, tr, qy, qz, out, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "transform kernels");
}

static tpc_status check_rans_params(const tpc_rans_params *p) {
    if (!p) return fail(TPC_ERR_ARG, "null rANS parameters");
    if (p->scale_bits < 1 || p->scale_bits > 16) return fail(TPC_ERR_ARG, "scale_bits outside 1..16");
    if (p->block_symbols < TPC_RANS_LANES || p->block_symbols % TPC_RANS_LANES || p->block_symbols > (1 << 24))
        return fail(TPC_ERR_ARG, "block_symbols must be a multiple of 64 in 64..2^24");
    return TPC_OK;
}

tpc_status tpc_rans_workspace_bytes(int64_t n, const tpc_rans_params *p, size_t *bytes) {
    g_err[0] = 0;
    tpc_status s = check_rans_params(p);
    if (s) return s;
    if (!bytes) return fail(TPC_ERR_ARG, "null bytes");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(TPC_ERR_ARG, "n outside 0..2^31-1");
    *bytes = rans_ws_layout(nullptr, n, p->block_symbols, nullptr);
    return TPC_OK;
}

tpc_status tpc_rans_max_bytes(int64_t n, int64_t range, const tpc_rans_params *p, size_t *bytes) {
    g_err[0] = 0;
    tpc_status s = check_rans_params(p);
    if (s) return s;
    if (!bytes) return fail(TPC_ERR_ARG, "null bytes");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(TPC_ERR_ARG, "n outside 0..2^31-1");
    if (range < 0 || range > TPC_RANS_MAX_RANGE) return fail(TPC_ERR_ARG, "range outside 0..2^20");
    const int64_t nb = n > 0 ? (n + p->block_symbols - 1) / p->block_symbols : 0;
    // the compressed table: at most 6 bytes for each of at most min(range, 2^16)
    // present symbols, padded to 4
    const int64_t d = n > 0 ? (range < 65536 ? range : 65536) : 0;
    *bytes = (size_t)(40 + ((6 * d + 3) & ~(int64_t)3) + 4 * (nb + 1) + 4 * TPC_RANS_LANES * nb + 2 * n);
    return TPC_OK;
}

tpc_status tpc_rans_encode(const int32_t *sym, int64_t n, const tpc_rans_params *p, void *out,
                           size_t out_cap, uint64_t *out_size, int32_t *dev_status, void *ws,
                           size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_rans_params(p);
    if (s) return s;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(TPC_ERR_ARG, "n outside 0..2^31-1");
    if (n > 0 && !sym) return fail(TPC_ERR_ARG, "null symbols");
    if (!out || !out_size || !dev_status) return fail(TPC_ERR_ARG, "null output, size or status");
    if (((uintptr_t)out & 3) != 0) return fail(TPC_ERR_ARG, "output not 4-byte aligned");
    if ((s = check_ws(ws, ws_bytes, rans_ws_layout(nullptr, n, p->block_symbols, nullptr)))) return s;
    RansJob J{sym, n, nullptr, (uint8_t *)out, (uint64_t)out_cap, out_size, dev_status};
    hipError_t e = launch_rans_batch(1, &J, p->scale_bits, p->block_symbols, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "rANS kernels");
}

static tpc_status check_rans_jobs(int32_t count, const tpc_rans_job *jobs, bool outputs) {
    if (count < 1 || count > TPC_RANS_BATCH_MAX) return fail(TPC_ERR_ARG, "count outside 1..%d", TPC_RANS_BATCH_MAX);
    if (!jobs) return fail(TPC_ERR_ARG, "null jobs");
    for (int k = 0; k < count; ++k) {
        const tpc_rans_job &J = jobs[k];
        if (J.n < 0 || J.n >= ((int64_t)1 << 31)) return fail(TPC_ERR_ARG, "job %d: n outside 0..2^31-1", k);
        if (!outputs) continue;
        if (J.n > 0 && !J.symbols) return fail(TPC_ERR_ARG, "job %d: null symbols", k);
        if (!J.out || !J.out_size || !J.dev_status) return fail(TPC_ERR_ARG, "job %d: null output, size or status", k);
        if (((uintptr_t)J.out & 3) != 0) return fail(TPC_ERR_ARG, "job %d: output not 4-byte aligned", k);
    }
    return TPC_OK;
}

static void rans_jobs(int32_t count, const tpc_rans_job *jobs, RansJob *J) {
    for (int k = 0; k < count; ++k)
        J[k] = RansJob{jobs[k].symbols, jobs[k].n, jobs[k].n_device, (uint8_t *)jobs[k].out,
                       (uint64_t)jobs[k].out_cap, jobs[k].out_size, jobs[k].dev_status};
}

tpc_status tpc_rans_batch_workspace_bytes(int32_t count, const tpc_rans_job *jobs, const tpc_rans_params *p,
                                          size_t *bytes) {
    g_err[0] = 0;
    tpc_status s = check_rans_params(p);
    if (s) return s;
    if (!bytes) return fail(TPC_ERR_ARG, "null bytes");
    if ((s = check_rans_jobs(count, jobs, false))) return s;
    RansJob J[TPC_RANS_BATCH_MAX];
    rans_jobs(count, jobs, J);
    *bytes = rans_batch_ws_bytes(count, J, p->block_symbols);
    return TPC_OK;
}

tpc_status tpc_rans_encode_batch(int32_t count, const tpc_rans_job *jobs, const tpc_rans_params *p, void *ws,
                                 size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    tpc_status s = check_rans_params(p);
    if (s) return s;
    if ((s = check_rans_jobs(count, jobs, true))) return s;
    RansJob J[TPC_RANS_BATCH_MAX];
    rans_jobs(count, jobs, J);
    if ((s = check_ws(ws, ws_bytes, rans_batch_ws_bytes(count, J, p->block_symbols)))) return s;
    hipError_t e = launch_rans_batch(count, J, p->scale_bits, p->block_symbols, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "rANS kernels");
}

tpc_status tpc_rans_decode_workspace_bytes(size_t *bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(TPC_ERR_ARG, "null bytes");
    *bytes = rans_decode_ws_bytes();
    return TPC_OK;
}

tpc_status tpc_rans_decode(const void *in, size_t size, int32_t *symbols, int64_t cap, int64_t *n_out,
                           int32_t *dev_status, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (!in || !n_out || !dev_status) return fail(TPC_ERR_ARG, "null stream, count or status");
    if (((uintptr_t)in & 3) != 0) return fail(TPC_ERR_ARG, "stream not 4-byte aligned");
    if (cap < 0 || cap >= ((int64_t)1 << 31)) return fail(TPC_ERR_ARG, "cap outside 0..2^31-1");
    if (cap > 0 && !symbols) return fail(TPC_ERR_ARG, "null symbols");
    tpc_status s = check_ws(ws, ws_bytes, rans_decode_ws_bytes());
    if (s) return s;
    hipError_t e = launch_rans_decode(in, (uint64_t)size, symbols, cap, n_out, dev_status, ws, (hipStream_t)stream);
    return e == hipSuccess ? TPC_OK : hip_fail(e, "rANS decoder kernels");
}

int32_t tpc_persistent_grid(const tpc_context *ctx) { return ctx ? ctx->persist_grid : 0; }

}  // extern "C"
