// Track following (gfx950): every seed is fitted, prolonged inwards and
// outwards with cluster pickup across up to max_miss empty pad rows, refitted
// over all its hits, and tracks that share most of their clusters with a
// longer one are marked as duplicates.
//
//  fl_index        workgroup per (frame, sector, row): the row's clusters in
//                  y cells (about one cluster per cell, counting sort with
//                  atomics in global memory); non-finite clusters are left out
//                  (they can never pass the gate)
//  fl_tracks       thread per seed, double precision throughout: seed fit
//                  (the seed's hits at the rows that hold them, so seeds may
//                  skip rows), inward prolongation, outward refit and
//                  prolongation, final refit; the search in a row scans only
//                  the cells covering the y extent of the gate ellipse
//  fl_owner_init   owner key of every cluster := none
//  fl_claim        thread per refitted track: 64-bit atomicMin of its key
//                  (n_rows - n_hits, index) on each of its clusters
//  fl_keep         thread per refitted track: duplicate if it owns fewer than
//                  half of its clusters
#include "tpc_fit_common.hpp"

#define TPC_TAN10 0.17632698070846498   // tan 10 deg: a pad row spans |y| <= x tan 10 deg

namespace {

struct FlIndex {
    float2 *grid;                 // [NR] (y0, cells per cm) of the segment's y cells
    int32_t *cstart;              // [N + NR] cell starts of segment s at row_offsets[s] + s (n + 1 entries)
    int32_t *cur;                 // [N + NR] scatter cursors
    float2 *syz;                  // [N] (y, z) ordered by cell within each segment
    int32_t *sid;                 // [N] their global ids
    float2 *yz;                   // [N] (y, z) by global id: one gather per hit
    unsigned long long *owner;    // [N] smallest key of a track holding the cluster
};

struct FlArgs {
    FitArgs F;                    // seeds, clusters, constants, outputs
    const int32_t *row_offsets;
    const int32_t *frame;         // [cap_seeds] frame of each seed
    int32_t n_frames;
    FlIndex X;
    int32_t *rows;                // [cap_seeds][n_rows] cluster per pad row, -1 for none
    double kbz;                   // -c Bz in double precision
    double gate;
    int32_t max_miss;
};

__device__ inline int ycell(float y, float y0, float iw, int n) {
    float c = (y - y0) * iw;
    c = fmaxf(c, 0.f);
    c = fminf(c, (float)(n - 1));
    return (int)c;
}

__global__ void __launch_bounds__(TPC_BLOCK)
fl_index(const int32_t *__restrict__ off, const float *__restrict__ y, const float *__restrict__ z,
         FlIndex X) {
    __shared__ float red[2][TPC_BLOCK / TPC_WAVE];
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    __shared__ int carry;
    const int seg = xcd_item(blockIdx.x, gridDim.x);
    const int a = off[seg], n = off[seg + 1] - a;
    const int base = a + seg;
    const int lane = threadIdx.x & (TPC_WAVE - 1), wid = threadIdx.x / TPC_WAVE;
    float lo = INFINITY, hi = -INFINITY;
    for (int j = threadIdx.x; j < n; j += TPC_BLOCK) {
        const float v = y[a + j], w = z[a + j];
        X.yz[a + j] = make_float2(v, w);
        if (isfinite(v) && isfinite(w)) {
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane == 0) {
        red[0][wid] = lo;
        red[1][wid] = hi;
    }
    for (int j = threadIdx.x; j <= n; j += TPC_BLOCK) X.cstart[base + j] = 0;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < TPC_BLOCK / TPC_WAVE; ++w) {
        lo = fminf(lo, red[0][w]);
        hi = fmaxf(hi, red[1][w]);
    }
    const float iw = hi > lo ? (float)n / (hi - lo) : 0.f;
    const float y0 = hi >= lo ? lo : 0.f;
    if (threadIdx.x == 0) X.grid[seg] = make_float2(y0, iw);
    for (int j = threadIdx.x; j < n; j += TPC_BLOCK) {
        const float v = y[a + j], w = z[a + j];
        if (isfinite(v) && isfinite(w)) atomicAdd(&X.cstart[base + ycell(v, y0, iw, n)], 1);
    }
    __syncthreads();
    for (int c0 = 0; c0 <= n; c0 += TPC_BLOCK) {
        const int j = c0 + threadIdx.x;
        const int v = j <= n ? X.cstart[base + j] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, sh, &tot);
        const int cr = carry;
        if (j <= n) {
            X.cstart[base + j] = cr + ex;
            X.cur[base + j] = cr + ex;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = cr + tot;
        __syncthreads();
    }
    for (int j = threadIdx.x; j < n; j += TPC_BLOCK) {
        const float v = y[a + j], w = z[a + j];
        if (isfinite(v) && isfinite(w)) {
            const int pos = atomicAdd(&X.cur[base + ycell(v, y0, iw, n)], 1);
            X.syz[a + pos] = make_float2(v, w);
            X.sid[a + pos] = a + j;
        }
    }
}

// The pad rows of the tracks of one workgroup (one wavefront, lane t works
// on track t) in LDS: row r of lane t at r * 64 + (t ^ (r & 31)).  A lane
// reading its own rows and the workgroup copying whole tracks out
// (consecutive lanes on consecutive rows) both meet distinct banks.
struct Strip {
    int32_t *s;
    int t;
    __device__ int32_t get(int r) const { return s[r * TPC_WAVE + (t ^ (r & 31))]; }
    __device__ void set(int r, int32_t v) const { s[r * TPC_WAVE + (t ^ (r & 31))] = v; }
};

// Cluster index data of one pad row segment, loaded a row ahead.
struct RowSeg {
    int a, n;
    float2 g;
    float x;
};

__device__ inline RowSeg row_seg(const FlArgs &A, int seg, int r) {
    RowSeg s;
    s.a = A.row_offsets[seg];
    s.n = A.row_offsets[seg + 1] - s.a;
    s.g = A.X.grid[seg];
    s.x = A.F.row_x[r];
    return s;
}

// Cluster of segment `seg` with the smallest predicted-residual chi2 against
// (p, C), ties to the smaller id; -1 if none is within the gate.  Only the
// cells covering the gate ellipse's y extent, sqrt(gate * S_yy), are read,
// widened so that float rounding of the bounds cannot exclude a cluster.
__device__ inline int pick_cluster(const FlArgs &A, int seg, const RowSeg &rs, const double p[5],
                                   const SymT<double> &C, float2 &yz) {
    const int a = rs.a, n = rs.n;
    if (n <= 0) return -1;
    const double S00 = C.c00 + A.F.vy, S01 = C.c10, S11 = C.c11 + A.F.vz;
    const double det = S00 * S11 - S01 * S01;
    if (!(det > 0.0)) return -1;
    const double idet = 1.0 / det;
    const double i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
    const double hy = sqrt(A.gate * S00) * (1.0 + 1e-6) + 1e-5 * (1.0 + fabs(p[0]));
    const int c0 = ycell((float)(p[0] - hy), rs.g.x, rs.g.y, n);
    const int c1 = ycell((float)(p[0] + hy), rs.g.x, rs.g.y, n);
    const int base = a + seg;
    const int j0 = A.X.cstart[base + c0], j1 = A.X.cstart[base + c1 + 1];
    int best = -1;
    double bchi = 0.0;
    for (int j = j0; j < j1; ++j) {
        const float2 c = A.X.syz[a + j];
        const int id = A.X.sid[a + j];
        const double r0 = (double)c.x - p[0], r1 = (double)c.y - p[1];
        const double chi = r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1);
        if (chi <= A.gate && (best < 0 || chi < bchi || (chi == bchi && id < best))) {
            best = id;
            bchi = chi;
            yz = c;
        }
    }
    return best;
}

__device__ inline void start_cov(const FitArgs &F, SymT<double> &C) {
    C = SymT<double>{};
    C.c00 = F.vy;
    C.c11 = F.vz;
    C.c22 = F.var_s;
    C.c33 = F.var_t;
    C.c44 = F.var_w;
}

// One prolongation row: helix step to the row's plane, stop (false) if it
// fails or leaves the row's width; pick = cluster taken up (state updated)
// or -1.
__device__ inline bool follow_row(const FlArgs &A, int seg, const RowSeg &rs, double p[5],
                                  SymT<double> &C, double &xcur, int &pick) {
    pick = -1;
    StepJac J;
    const double xr = (double)rs.x;
    if (!helix_step<double, double>(p, xr - xcur, A.kbz, A.F.max_sin, J)) return false;
    sym_transport<double, false>(C, J);
    xcur = xr;
    if (!(fabs(p[0]) <= xr * TPC_TAN10)) return false;
    float2 yz;
    const int c = pick_cluster(A, seg, rs, p, C, yz);
    if (c < 0) return true;
    const double dchi = kalman_update<double>(p, C, (double)yz.x, (double)yz.y, A.F.vy, A.F.vz);
    const double chk = dchi + p[0] + p[1] + p[2] + p[3] + p[4];
    if (!(chk - chk == 0.0)) return false;
    pick = c;
    return true;
}

// Prolongation from the row after `from` in direction dir (-1 inwards, +1
// outwards) until a stop or more than max_miss empty rows in a row; the
// cluster taken in each row goes to the strip; returns the last row with a
// cluster (`from` if none) and counts the clusters taken.
__device__ inline int prolong(const FlArgs &A, const Strip &S, int seg0, int from, int dir, double p[5],
                              SymT<double> &C, double &xcur, double plast[5], int &taken) {
    const int R = A.F.n_rows;
    int last = from, miss = 0;
    int r = from + dir;
    if (r < 0 || r >= R) return last;
    RowSeg nx = row_seg(A, seg0 + r, r);
    for (; r >= 0 && r < R; r += dir) {
        const RowSeg cs = nx;
        const int rn = r + dir;
        if (rn >= 0 && rn < R) nx = row_seg(A, seg0 + rn, rn);      // one row ahead
        int pick;
        if (!follow_row(A, seg0 + r, cs, p, C, xcur, pick)) break;
        if (pick >= 0) {
            S.set(r, pick);
            last = r;
            miss = 0;
            ++taken;
            for (int q = 0; q < 5; ++q) plast[q] = p[q];
        } else if (++miss > A.max_miss) {
            break;
        }
    }
    return last;
}

// Inward fit of the hits of rows lo..hi (m of them; -1 = no hit): three-point
// start at the outermost, middle ((m - 1) / 2 in ascending row order) and
// innermost hits, then a helix step and Kalman update per hit.  The next
// hit's plane and coordinates are loaded a step ahead.
__device__ inline int fit_rows(const FlArgs &A, const Strip &S, int lo, int hi, int m, double p[5],
                               SymT<double> &C, double &chi2, double &xcur) {
    const FitArgs &F = A.F;
    chi2 = 0.0;
    xcur = (double)F.row_x[hi];
    start_cov(F, C);
    for (int q = 0; q < 5; ++q) p[q] = 0.0;
    if (m < 3) return TPC_FIT_INIT_FAIL;
    int mid = lo;
    for (int r = lo, k = 0, want = (m - 1) / 2; r <= hi; ++r) {
        if (S.get(r) < 0) continue;
        if (k == want) {
            mid = r;
            break;
        }
        ++k;
    }
    const float2 ha = A.X.yz[S.get(hi)], hb = A.X.yz[S.get(mid)], hc = A.X.yz[S.get(lo)];
    if (!helix_start<double, double>((double)F.row_x[hi], (double)ha.x, (double)ha.y,
                                     (double)F.row_x[mid], (double)hb.x, (double)F.row_x[lo],
                                     (double)hc.x, (double)hc.y, A.kbz, F.max_sin, p))
        return TPC_FIT_INIT_FAIL;
    int r = hi - 1;
    while (r >= lo && S.get(r) < 0) --r;
    int id = r >= lo ? S.get(r) : S.get(hi);
    float2 hk = A.X.yz[id];
    float xk = F.row_x[r >= lo ? r : hi];
    while (r >= lo) {
        int rn = r - 1;
        while (rn >= lo && S.get(rn) < 0) --rn;
        const int idn = rn >= lo ? S.get(rn) : id;
        const float2 hn = A.X.yz[idn];
        const float xn = F.row_x[rn >= lo ? rn : r];
        const float yk = hk.x, zk = hk.y;
        StepJac J;
        const bool stepped = helix_step<double, double>(p, (double)xk - xcur, A.kbz, F.max_sin, J);
        sym_transport<double, false>(C, J);
        const double dchi = kalman_update<double>(p, C, (double)yk, (double)zk, F.vy, F.vz);
        chi2 += dchi;
        const double chk = chi2 + p[0] + p[1] + p[2] + p[3] + p[4];
        if (!stepped) return TPC_FIT_SIN_FAIL;
        if (!(dchi >= 0.0) || !(chk - chk == 0.0)) return TPC_FIT_NUM_FAIL;
        xcur = (double)xk;
        r = rn;
        id = idn;
        hk = hn;
        xk = xn;
    }
    return TPC_FIT_OK;
}

// Outward filter from the innermost hit (row lo) through the hits up to row
// hi, from a restart state: y, z of the hit at lo, the other parameters as
// given, the start covariance.  False if a step or update fails.
__device__ inline bool filter_out(const FlArgs &A, const Strip &S, int lo, int hi, double p[5],
                                  SymT<double> &C, double &xcur) {
    const FitArgs &F = A.F;
    const int i0 = S.get(lo);
    const float2 h0 = A.X.yz[i0];
    p[0] = (double)h0.x;
    p[1] = (double)h0.y;
    start_cov(F, C);
    xcur = (double)F.row_x[lo];
    int r = lo + 1;
    while (r <= hi && S.get(r) < 0) ++r;
    int id = r <= hi ? S.get(r) : i0;
    float2 hk = A.X.yz[id];
    float xk = F.row_x[r <= hi ? r : lo];
    while (r <= hi) {
        int rn = r + 1;
        while (rn <= hi && S.get(rn) < 0) ++rn;
        const int idn = rn <= hi ? S.get(rn) : id;
        const float2 hn = A.X.yz[idn];
        const float xn = F.row_x[rn <= hi ? rn : r];
        const float yk = hk.x, zk = hk.y;
        StepJac J;
        if (!helix_step<double, double>(p, (double)xk - xcur, A.kbz, F.max_sin, J)) return false;
        sym_transport<double, false>(C, J);
        xcur = (double)xk;
        const double dchi = kalman_update<double>(p, C, (double)yk, (double)zk, F.vy, F.vz);
        const double chk = dchi + p[0] + p[1] + p[2] + p[3] + p[4];
        if (!(dchi >= 0.0) || !(chk - chk == 0.0)) return false;
        r = rn;
        id = idn;
        hk = hn;
        xk = xn;
    }
    return true;
}

__device__ inline void write_track(const FitArgs &F, int i, double xcur, const double p[5],
                                   const SymT<double> &C, double chi2, int m, int status) {
    F.out.x[i] = (float)xcur;
    float *po = F.out.par + (size_t)i * 5;
    for (int q = 0; q < 5; ++q) po[q] = (float)p[q];
    float *co = F.out.cov + (size_t)i * 15;
    const double cc[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                           C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    for (int q = 0; q < 15; ++q) co[q] = (float)cc[q];
    F.out.chi2[i] = (float)chi2;
    F.out.ndf[i] = 2 * m - 5;
    F.out.status[i] = status;
}

// Places the seed's hits in the strip, each at the pad row of its (frame,
// sector) whose id range holds it (seeds from links across a missing row
// skip rows; first_row is not read): the outermost hit's row by binary
// search over the row starts ro[0 .. R], each next one by a walk down.
// False if a hit lies outside the (frame, sector) or the rows do not rise
// strictly (then the strip may hold some of the hits).
__device__ inline bool place_seed(const SeedView &sv, const int32_t *ro, int R, const Strip &S, int &lo,
                                  int &hi) {
    const int32_t top = sv.hh[sv.n - 1];
    if (top < ro[0] || top >= ro[R]) return false;
    int a = 0, b = R - 1;                          // ro[a] <= top < ro[b + 1]
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (ro[mid] <= top) a = mid;
        else b = mid - 1;
    }
    int r = a;
    hi = r;
    S.set(r, top);
    for (int k = sv.n - 2; k >= 0; --k) {
        const int32_t id = sv.hh[k];
        int q = r - 1;
        while (q >= 0 && ro[q] > id) --q;
        if (q < 0 || id >= ro[q + 1]) return false;
        r = q;
        S.set(r, id);
    }
    lo = r;
    return true;
}

__device__ inline void follow_one(const FlArgs &A, int i, const Strip &S) {
    const FitArgs &F = A.F;
    const SeedView sv = seed_view(F, i);
    const int R = F.n_rows;
    for (int r = 0; r < R; ++r) S.set(r, -1);
    double p[5] = {0, 0, 0, 0, 0};
    SymT<double> C = {};
    double chi2 = 0.0, xcur = 0.0;
    int m = sv.n;
    int lo = 0, hi = 0;
    // a seed list not written by tpc_ca_seed may hold anything
    bool ok = sv.n >= 3 && sv.o0 >= 0 && sv.o0 <= F.cap_hits - sv.n && sv.sec >= 0 && sv.sec < F.n_sectors &&
              (uint32_t)A.frame[i] < (uint32_t)A.n_frames;
    if (ok) {
        const int32_t *ro = A.row_offsets + ((size_t)A.frame[i] * F.n_sectors + sv.sec) * R;
        ok = place_seed(sv, ro, R, S, lo, hi);
    }
    if (!ok) {
        for (int r = 0; r < R; ++r) S.set(r, -1);
        write_track(F, i, 0.0, p, C, 0.0, sv.n, TPC_FIT_INIT_FAIL);
        return;
    }
    int status = fit_rows(A, S, lo, hi, m, p, C, chi2, xcur);
    // the seed fit is the result unless a cluster is taken up
    write_track(F, i, xcur, p, C, chi2, m, status);
    if (status != TPC_FIT_OK) return;
    const int seg0 = (A.frame[i] * F.n_sectors + sv.sec) * R;
    int taken = 0;
    double plo[5] = {p[0], p[1], p[2], p[3], p[4]};
    lo = prolong(A, S, seg0, lo, -1, p, C, xcur, plo, taken);
    // outwards only where there are rows above the outermost hit (the
    // outward filter's state is used for nothing else)
    if (hi < R - 1) {
        for (int q = 2; q < 5; ++q) p[q] = plo[q];
        if (filter_out(A, S, lo, hi, p, C, xcur)) hi = prolong(A, S, seg0, hi, +1, p, C, xcur, plo, taken);
    }
    if (taken == 0) return;
    m = 0;
    for (int r = lo; r <= hi; ++r) m += S.get(r) >= 0;
    status = fit_rows(A, S, lo, hi, m, p, C, chi2, xcur);
    write_track(F, i, xcur, p, C, chi2, m, status);
}

// One wavefront per workgroup; lane t follows seed i0 + t of each round,
// then the workgroup writes the round's rows out row-contiguously.
__global__ void __launch_bounds__(TPC_WAVE)
fl_tracks(FlArgs A) {
    extern __shared__ int32_t fl_strip[];
    const int t = threadIdx.x;
    const int R = A.F.n_rows;
    const Strip S{fl_strip, t};
    int T = *A.F.n_seeds;
    if (T > A.F.cap_seeds) T = A.F.cap_seeds;
    // blocks with work, renumbered so that each XCD takes consecutive seeds
    // (one sector's seeds and clusters then stay in one L2)
    int G = (T + TPC_WAVE - 1) / TPC_WAVE;
    G = G < (int)gridDim.x ? G : (int)gridDim.x;
    if ((int)blockIdx.x >= G) return;
    for (int i0 = xcd_item(blockIdx.x, G) * TPC_WAVE; i0 < T; i0 += G * TPC_WAVE) {
        if (i0 + t < T) follow_one(A, i0 + t, S);
        __syncthreads();
        const int nt = T - i0 < TPC_WAVE ? T - i0 : TPC_WAVE;
        int32_t *out = A.rows + (size_t)i0 * R;
        for (int e = t; e < nt * R; e += TPC_WAVE) {
            const int u = e / R, r = e - u * R;
            out[e] = fl_strip[r * TPC_WAVE + (u ^ (r & 31))];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
fl_owner_init(unsigned long long *__restrict__ owner, int32_t N) {
    for (int c = blockIdx.x * TPC_BLOCK + threadIdx.x; c < N; c += gridDim.x * TPC_BLOCK) owner[c] = ~0ull;
}

__device__ inline unsigned long long track_key(int n_rows, int ndf, int i) {
    return ((unsigned long long)(uint32_t)(n_rows - (ndf + 5) / 2) << 32) | (uint32_t)i;
}

// Ownership passes: one wavefront per track, lanes on consecutive rows.
__global__ void __launch_bounds__(TPC_BLOCK)
fl_claim(const int32_t *__restrict__ n_seeds, int32_t cap_seeds, int32_t n_rows,
         const int32_t *__restrict__ rows, const int32_t *__restrict__ status,
         const int32_t *__restrict__ ndf, unsigned long long *__restrict__ owner) {
    int T = *n_seeds;
    if (T > cap_seeds) T = cap_seeds;
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    constexpr int WB = TPC_BLOCK / TPC_WAVE;
    int G = (T + WB - 1) / WB;
    G = G < (int)gridDim.x ? G : (int)gridDim.x;
    if ((int)blockIdx.x >= G) return;
    for (int i = xcd_item(blockIdx.x, G) * WB + threadIdx.x / TPC_WAVE; i < T; i += G * WB) {
        if (status[i] != TPC_FIT_OK) continue;
        const unsigned long long key = track_key(n_rows, ndf[i], i);
        const int32_t *rw = rows + (size_t)i * n_rows;
        for (int r = lane; r < n_rows; r += TPC_WAVE) {
            const int c = rw[r];
            if (c >= 0) atomicMin(&owner[c], key);
        }
    }
}

__global__ void __launch_bounds__(TPC_BLOCK)
fl_keep(const int32_t *__restrict__ n_seeds, int32_t cap_seeds, int32_t n_rows,
        const int32_t *__restrict__ rows, int32_t *__restrict__ status, const int32_t *__restrict__ ndf,
        const unsigned long long *__restrict__ owner) {
    int T = *n_seeds;
    if (T > cap_seeds) T = cap_seeds;
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    constexpr int WB = TPC_BLOCK / TPC_WAVE;
    int G = (T + WB - 1) / WB;
    G = G < (int)gridDim.x ? G : (int)gridDim.x;
    if ((int)blockIdx.x >= G) return;
    for (int i = xcd_item(blockIdx.x, G) * WB + threadIdx.x / TPC_WAVE; i < T; i += G * WB) {
        if (status[i] != TPC_FIT_OK) continue;
        const unsigned long long key = track_key(n_rows, ndf[i], i);
        const int32_t *rw = rows + (size_t)i * n_rows;
        int owned = 0;
        for (int r0 = 0; r0 < n_rows; r0 += TPC_WAVE) {
            const int r = r0 + lane;
            const int c = r < n_rows ? rw[r] : -1;
            owned += __popcll(__ballot(c >= 0 && owner[c] == key));
        }
        if (lane == 0 && 2 * owned < (ndf[i] + 5) / 2) status[i] = TPC_FOLLOW_DUPLICATE;
    }
}

int grid_for(int64_t items) {
    int64_t b = (items + TPC_BLOCK - 1) / TPC_BLOCK;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

size_t follow_ws_layout(void *ws, int64_t N, int64_t NR, void *out) {
    WsCarver w(ws);
    FlIndex X;
    X.grid = w.take<float2>(NR > 0 ? NR : 1);
    X.cstart = w.take<int32_t>(N + NR + 1);
    X.cur = w.take<int32_t>(N + NR + 1);
    X.syz = w.take<float2>(N > 0 ? N : 1);
    X.sid = w.take<int32_t>(N > 0 ? N : 1);
    X.yz = w.take<float2>(N > 0 ? N : 1);
    X.owner = w.take<unsigned long long>(N > 0 ? N : 1);
    if (out) *static_cast<FlIndex *>(out) = X;
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_follow(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                         double gate, int32_t max_miss, int32_t *rows, const tpc_tracks *tr,
                         void *ws, hipStream_t st) {
    const tpc_config &c = ctx->cfg;
    const int64_t NR = (int64_t)fr->n_frames * c.n_sectors * c.n_rows;
    FlArgs A;
    A.F = make_fit_args(ctx, fr, sd, nullptr);
    A.F.out = *tr;
    A.row_offsets = fr->row_offsets;
    A.frame = sd->frame;
    A.n_frames = fr->n_frames;
    follow_ws_layout(ws, fr->n_clusters, NR, &A.X);
    A.rows = rows;
    A.kbz = -0.00299792458 * (double)c.bz;
    A.gate = gate;
    A.max_miss = max_miss;
    hipLaunchKernelGGL(fl_index, dim3((unsigned)NR), dim3(TPC_BLOCK), 0, st, fr->row_offsets, fr->y,
                       fr->z, A.X);
    int tb = (int)((sd->cap_seeds + TPC_WAVE - 1) / TPC_WAVE);
    tb = tb > 16384 ? 16384 : (tb < 1 ? 1 : tb);
    hipLaunchKernelGGL(fl_tracks, dim3(tb), dim3(TPC_WAVE), (size_t)c.n_rows * TPC_WAVE * sizeof(int32_t), st, A);
    hipLaunchKernelGGL(fl_owner_init, dim3(grid_for(fr->n_clusters)), dim3(TPC_BLOCK), 0, st, A.X.owner,
                       fr->n_clusters);
    const int wb = grid_for((int64_t)sd->cap_seeds * TPC_WAVE);
    hipLaunchKernelGGL(fl_claim, dim3(wb), dim3(TPC_BLOCK), 0, st, sd->n_seeds,
                       sd->cap_seeds, c.n_rows, rows, tr->status, tr->ndf, A.X.owner);
    hipLaunchKernelGGL(fl_keep, dim3(wb), dim3(TPC_BLOCK), 0, st, sd->n_seeds,
                       sd->cap_seeds, c.n_rows, rows, tr->status, tr->ndf, A.X.owner);
    return hipGetLastError();
}
