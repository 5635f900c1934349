// Per-seed access shared by the fit and its adjoint.
#pragma once

#include "tpc_fit_math.hpp"
#include "tpc_internal.hpp"

#define TPC_CKPT_WORDS 20      // doubles per checkpoint: p[5], covariance lower triangle[15]

struct FitArgs {
    const int32_t *offsets, *hits, *sector, *first_row, *n_seeds;
    int32_t cap_seeds, cap_hits;
    const float *y, *z, *row_x, *map;
    const float2 *hyz;     // (y, z) of every seed hit in seed-hit order, or null
    int32_t n_rows, n_sectors, n_clusters;
    float kbz, max_sin;
    double vy, vz, var_s, var_t, var_w;
    double *ckpt;
    int32_t ckpt_rows;
    tpc_tracks out;
    const int32_t *order;      // optional: fit seeds order[0 .. *n_order) instead of 0 .. T
    const int32_t *n_order;
};

struct SeedView {
    int32_t o0, n, row0, sec;
    bool sane;
    const int32_t *hh;     // hit ids of the seed
    const float *mp;       // map rows of the seed's sector, or null
};

// A seed from tpc_ca_seed always passes these checks; others are flagged
// instead of being read out of bounds.
__host__ __device__ inline SeedView seed_view(const FitArgs &A, int i) {
    SeedView v;
    v.o0 = A.offsets[i];
    v.n = A.offsets[i + 1] - v.o0;
    v.row0 = A.first_row[i];
    v.sec = A.sector[i];
    v.sane = v.n >= 3 && v.row0 >= 0 && v.row0 + v.n <= A.n_rows && v.sec >= 0 &&
             v.sec < A.n_sectors && v.o0 >= 0 && v.o0 <= A.cap_hits - v.n;
    v.hh = A.hits + v.o0;
    v.mp = (A.map && v.sane) ? A.map + (size_t)v.sec * A.n_rows * 2 : nullptr;
    return v;
}

// Raw (y, z) of hit k of the seed (global id `id`): from the seed-ordered
// copy when there is one (contiguous per seed, no id indirection).
__host__ __device__ inline float2 hit_raw(const FitArgs &A, const SeedView &v, int k, int32_t id) {
    if (A.hyz) return A.hyz[v.o0 + k];
    const uint32_t NC = (uint32_t)A.n_clusters;
    const int32_t j = (uint32_t)id < NC ? id : 0;
    return make_float2(A.y[j], A.z[j]);
}

// Corrected measurement of hit k in double precision.
__host__ __device__ inline void hit_fix(const FitArgs &A, const SeedView &v, int k, float2 raw,
                                        double &my, double &mz) {
    my = (double)raw.x;
    mz = (double)raw.y;
    if (v.mp) {
        my -= (double)v.mp[(v.row0 + k) * 2];
        mz -= (double)v.mp[(v.row0 + k) * 2 + 1];
    }
}

__host__ __device__ inline void hit_meas(const FitArgs &A, const SeedView &v, int k, int32_t id, double &my,
                                         double &mz) {
    hit_fix(A, v, k, hit_raw(A, v, k, id), my, mz);
}

__host__ __device__ inline bool start_state(const FitArgs &A, const SeedView &v, const float *xs, double p[5]) {
    const int ka = v.n - 1, kb = (v.n - 1) / 2;
    double ya, za, yb, zb, yc, zc;
    hit_meas(A, v, ka, A.hyz ? 0 : v.hh[ka], ya, za);
    hit_meas(A, v, kb, A.hyz ? 0 : v.hh[kb], yb, zb);
    hit_meas(A, v, 0, A.hyz ? 0 : v.hh[0], yc, zc);
    (void)zb;
    return helix_start<double>(xs[v.row0 + ka], ya, za, xs[v.row0 + kb], yb, xs[v.row0], yc, zc,
                               A.kbz, A.max_sin, p);
}

// Checkpoint slots: track i with hit offset o0 owns slots o0/K + i .. + ceil(n/K);
// slots of consecutive tracks never overlap.
__host__ __device__ inline int64_t ckpt_slot(int32_t o0, int32_t i, int32_t K) {
    return (int64_t)(o0 / K) + i;
}

__host__ __device__ inline void write_ckpt(double *ck, const double p[5], const SymT<double> &C) {
#pragma unroll
    for (int q = 0; q < 5; ++q) ck[q] = p[q];
    ck[5] = C.c00; ck[6] = C.c10; ck[7] = C.c11; ck[8] = C.c20; ck[9] = C.c21;
    ck[10] = C.c22; ck[11] = C.c30; ck[12] = C.c31; ck[13] = C.c32; ck[14] = C.c33;
    ck[15] = C.c40; ck[16] = C.c41; ck[17] = C.c42; ck[18] = C.c43; ck[19] = C.c44;
}

__host__ __device__ inline void read_ckpt(const double *ck, double p[5], SymT<double> &C) {
#pragma unroll
    for (int q = 0; q < 5; ++q) p[q] = ck[q];
    C.c00 = ck[5]; C.c10 = ck[6]; C.c11 = ck[7]; C.c20 = ck[8]; C.c21 = ck[9];
    C.c22 = ck[10]; C.c30 = ck[11]; C.c31 = ck[12]; C.c32 = ck[13]; C.c33 = ck[14];
    C.c40 = ck[15]; C.c41 = ck[16]; C.c42 = ck[17]; C.c43 = ck[18]; C.c44 = ck[19];
}

// Forward fit of seed i (one thread's work); xs = row table.
__host__ __device__ inline void fit_one(const FitArgs &A, int i, const float *xs) {
    SeedView sv = seed_view(A, i);
    double p[5] = {0, 0, 0, 0, 0};
    SymT<double> C = {};
    double chi2 = 0.0;
    int status = TPC_FIT_OK;
    float xcur = sv.sane ? xs[sv.row0 + sv.n - 1] : 0.0f;
    if (!sv.sane || !start_state(A, sv, xs, p)) status = TPC_FIT_INIT_FAIL;
    C.c00 = A.vy;
    C.c11 = A.vz;
    C.c22 = A.var_s;
    C.c33 = A.var_t;
    C.c44 = A.var_w;
    double *ck = A.ckpt ? A.ckpt + (size_t)ckpt_slot(sv.o0, i, A.ckpt_rows) * TPC_CKPT_WORDS : nullptr;
    if (status == TPC_FIT_OK) {
        if (ck) write_ckpt(ck, p, C);
        // Each hit is read one step ahead, into the register its predecessor
        // has just been consumed from (no copy at the loop edge, so the load
        // is waited for only at its use a whole step later).
        float2 raw = hit_raw(A, sv, sv.n - 2, A.hyz ? 0 : sv.hh[sv.n - 2]);
        float xk = xs[sv.row0 + sv.n - 2];            // plane of hit k
        // the covariance half of each update is applied at the next step,
        // beside its helix step (G is zero before the first update)
        Gain<double> G = {};
        for (int k = sv.n - 2, j = 1; k >= 0; --k, ++j) {
            double my, mz;
            hit_fix(A, sv, k, raw, my, mz);
            const float xnext = k > 0 ? xs[sv.row0 + k - 1] : 0.0f;
            if (k > 0) raw = hit_raw(A, sv, k - 1, A.hyz ? 0 : sv.hh[k - 1]);
            // one exit test per step: the step and the update are evaluated
            // unconditionally and a failed track's final state is not used
            kalman_cov(C, G);
            StepJac J;
            const bool stepped = helix_step(p, xk - xcur, A.kbz, A.max_sin, J);
            sym_transport<double, false>(C, J);
            const double dchi = kalman_gain<double>(p, C, my, mz, A.vy, A.vz, G);
            chi2 += dchi;
            const double chk = chi2 + p[0] + p[1] + p[2] + p[3] + p[4];
            if (!stepped || !(dchi >= 0.0) || !(chk - chk == 0.0)) {   // non-finite state too
                status = stepped ? TPC_FIT_NUM_FAIL : TPC_FIT_SIN_FAIL;
                break;
            }
            xcur = xk;
            xk = xnext;
            // state after j updates opens segment j / K of the adjoint
            if (ck && j % A.ckpt_rows == 0 && k > 0) {
                SymT<double> Cj = C;
                kalman_cov(Cj, G);
                write_ckpt(ck + (size_t)(j / A.ckpt_rows) * TPC_CKPT_WORDS, p, Cj);
            }
        }
        kalman_cov(C, G);                             // the last update's covariance half
    }
    A.out.x[i] = xcur;
    float *po = A.out.par + (size_t)i * 5;
    for (int q = 0; q < 5; ++q) po[q] = (float)p[q];
    float *co = A.out.cov + (size_t)i * 15;
    const double cc[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                           C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    for (int q = 0; q < 15; ++q) co[q] = (float)cc[q];
    A.out.chi2[i] = (float)chi2;
    A.out.ndf[i] = 2 * sv.n - 5;
    A.out.status[i] = status;
}

// Tape of filter states before each step of one segment; word q of step s at
// tp[(s * TPC_CKPT_WORDS + q) * stride].
__host__ __device__ inline void tape_put(double *tp, int stride, int step, const double p[5],
                                         const SymT<double> &C) {
    double *b = tp + (size_t)step * TPC_CKPT_WORDS * stride;
    const double v[TPC_CKPT_WORDS] = {p[0], p[1], p[2], p[3], p[4], C.c00, C.c10, C.c11, C.c20, C.c21,
                                      C.c22, C.c30, C.c31, C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
#pragma unroll
    for (int q = 0; q < TPC_CKPT_WORDS; ++q) b[q * stride] = v[q];
}

__host__ __device__ inline void tape_get(const double *tp, int stride, int step, double p[5],
                                         SymT<double> &C) {
    const double *b = tp + (size_t)step * TPC_CKPT_WORDS * stride;
    double v[TPC_CKPT_WORDS];
#pragma unroll
    for (int q = 0; q < TPC_CKPT_WORDS; ++q) v[q] = b[q * stride];
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2]; p[3] = v[3]; p[4] = v[4];
    C.c00 = v[5]; C.c10 = v[6]; C.c11 = v[7]; C.c20 = v[8]; C.c21 = v[9]; C.c22 = v[10];
    C.c30 = v[11]; C.c31 = v[12]; C.c32 = v[13]; C.c33 = v[14]; C.c40 = v[15]; C.c41 = v[16];
    C.c42 = v[17]; C.c43 = v[18]; C.c44 = v[19];
}

// Reverse pass of seed i (one thread's work): writes dL/d(my, mz) for every
// hit of the seed into g[offsets[i] ..], zeros for a failed fit.
__host__ __device__ inline void adj_one(const FitArgs &F, const int32_t *status, const double *ckpt,
                                        float2 *gbuf, int i, const float *xs, double *tp, int stride) {
    const int K = F.ckpt_rows;
    const SeedView sv = seed_view(F, i);
    if (!sv.sane) return;
    float2 *g = gbuf + sv.o0;
    if (status[i] != TPC_FIT_OK) {
        for (int k = 0; k < sv.n; ++k) g[k] = make_float2(0.f, 0.f);
        return;
    }
    const int n = sv.n, nsteps = n - 1;
    const int nseg = (nsteps + K - 1) / K;
    const double *ck = ckpt + (size_t)ckpt_slot(sv.o0, i, K) * TPC_CKPT_WORDS;
    double pbar[5] = {0, 0, 0, 0, 0};
    SymT<double> Cbar = {};
    for (int c = nseg - 1; c >= 0; --c) {
        double p[5];
        SymT<double> C;
        read_ckpt(ck + (size_t)c * TPC_CKPT_WORDS, p, C);
        const int j0 = c * K;
        const int jend = j0 + K < nsteps ? j0 + K : nsteps;
        float xcur = xs[sv.row0 + n - 1 - j0];
        for (int j = j0 + 1; j <= jend; ++j) {          // recompute the segment, taping
            const int k = n - 1 - j;
            tape_put(tp, stride, j - j0 - 1, p, C);
            double my, mz;
            hit_meas(F, sv, k, F.hyz ? 0 : sv.hh[k], my, mz);
            const float xk = xs[sv.row0 + k];
            StepJac J;
            helix_step(p, xk - xcur, F.kbz, 2.0f, J);
            xcur = xk;
            sym_transport<double, false>(C, J);
            kalman_update<double>(p, C, my, mz, F.vy, F.vz);
        }
        for (int j = jend; j > j0; --j) {               // then run it backwards
            const int k = n - 1 - j;
            double pb[5];
            SymT<double> Cb;
            tape_get(tp, stride, j - j0 - 1, pb, Cb);
            double my, mz;
            hit_meas(F, sv, k, F.hyz ? 0 : sv.hh[k], my, mz);
            const float dx = xs[sv.row0 + k] - xs[sv.row0 + k + 1];
            double mby, mbz;
            step_adjoint<double>(pb, Cb, dx, F.kbz, my, mz, F.vy, F.vz, 1.0, pbar, Cbar, mby, mbz);
            g[k] = make_float2((float)mby, (float)mbz);
        }
    }
    // three-point start: hits A = n-1, B = (n-1)/2, C = 0
    const int ka = n - 1, kb = (n - 1) / 2;
    double ya, za, yb, zb, yc, zc;
    hit_meas(F, sv, ka, F.hyz ? 0 : sv.hh[ka], ya, za);
    hit_meas(F, sv, kb, F.hyz ? 0 : sv.hh[kb], yb, zb);
    hit_meas(F, sv, 0, F.hyz ? 0 : sv.hh[0], yc, zc);
    (void)zb;
    double bya, bza, byb, byc, bzc;
    start_adjoint<double>(xs[sv.row0 + ka], ya, za, xs[sv.row0 + kb], yb, xs[sv.row0], yc, zc, F.kbz,
                          pbar, bya, bza, byb, byc, bzc);
    g[ka] = make_float2((float)bya, (float)bza);
    const float2 gb = g[kb];
    g[kb] = make_float2(gb.x + (float)byb, gb.y);
    const float2 gc = g[0];
    g[0] = make_float2(gc.x + (float)byc, gc.y + (float)bzc);
}

FitArgs make_fit_args(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                      const float *map);
hipError_t launch_fit_args(const FitArgs &A, hipStream_t st, bool ordered = false, int block = 0,
                           int spt = 0);
