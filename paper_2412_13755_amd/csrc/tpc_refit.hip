// Tracks assembled from linked segments and refitted over all their hits
// (gfx950).  The links come from the merging kernels: next/prev join a
// particle's fitted segments across sector edges, leg joins the two legs of
// a looper.
//
//  rf_ids_init,    track ids: the connected components of the segments of
//  rf_ids_union,   status 0 under both kinds of link, each named by its
//  rf_ids_final    smallest segment (union-find in place in the output:
//                  a root is hooked under the smaller root by compare-and-
//                  swap, so every component's root ends as its minimum
//                  whatever the order; then every segment takes its root)
//  rf_chains       thread per chain head (a segment of status 0 with no
//                  counted prev link): the hits of the chain, head to tail,
//                  each in its own sector's frame; the exact circle through
//                  hits n-1, (n-1)/2 and 0 seen from the frame of hit n-1
//                  starts the filter there, which runs inwards: a helix
//                  step within a segment, the rotation into the next
//                  segment's frame and the step on to its plane across a
//                  boundary (covariance J C J^T), then the update.  FP64.
//  rf_loops        thread per looper leg pair (i < j): the circles of the
//                  two legs' refitted chains, fused in i's sense (the joint
//                  circle for the linearised problem, 4x4 Cholesky)
#include "tpc_fit_math.hpp"
#include "tpc_refit.hpp"

namespace {

#define RF_MAX_CHAIN 18          // one segment per sector of a side
#define RF_LEG_MAX_RADIUS 250.0

struct RfArgs {
    const int32_t *offsets, *hits, *sector, *first_row, *n_seeds;
    int32_t cap_seeds, cap_hits;
    const float *y, *z, *row_x, *map;
    int32_t n_rows, n_sectors, n_clusters;
    double kbz;
    float max_sin;
    double vy, vz, var_s, var_t, var_w;
    const int32_t *status, *next, *prev, *leg;
    int32_t *track_id;
    tpc_tracks out;
    float *loop_par, *loop_cov, *loop_chi2;
};

__device__ inline int rf_count(const RfArgs &A) {
    const int n = *A.n_seeds;
    return n < 0 ? 0 : (n < A.cap_seeds ? n : A.cap_seeds);
}

// Counted links (both ends of status 0, each end naming the other).
__device__ inline int next_link(const RfArgs &A, int T, int i) {
    const int j = A.next[i];
    return j >= 0 && j < T && j != i && A.prev[j] == i && A.status[i] == 0 && A.status[j] == 0 ? j : -1;
}
__device__ inline int prev_link(const RfArgs &A, int T, int i) {
    const int a = A.prev[i];
    return a >= 0 && a < T && a != i && A.next[a] == i && A.status[i] == 0 && A.status[a] == 0 ? a : -1;
}
__device__ inline int leg_link(const RfArgs &A, int T, int i) {
    if (!A.leg) return -1;
    const int j = A.leg[i];
    return j >= 0 && j < T && j != i && A.leg[j] == i && A.status[i] == 0 && A.status[j] == 0 ? j : -1;
}

__device__ inline double sector_angle(int sec, int n_sectors) {
    const double pi = 3.14159265358979323846;
    return n_sectors == 1 ? 0.0 : (double)(sec % 18) * (pi / 9.0) + pi / 18.0;
}

// ---------------------------------------------------------------------------
// track ids

__global__ void __launch_bounds__(TPC_BLOCK) rf_ids_init(RfArgs A) {
    const int T = rf_count(A);
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        A.track_id[i] = A.status[i] == 0 ? i : -1;
}

// Parents only ever point to smaller indices, so a root walk ends.
__device__ inline int uf_root(const int32_t *P, int x) {
    for (;;) {
        const int p = __atomic_load_n(P + x, __ATOMIC_RELAXED);
        if (p == x) return x;
        x = p;
    }
}

__device__ inline void uf_unite(int32_t *P, int a, int b) {
    for (;;) {
        a = uf_root(P, a);
        b = uf_root(P, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        // hook the larger root under the smaller; retry if it has moved
        if (atomicCAS(P + b, b, a) == b) return;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) rf_ids_union(RfArgs A) {
    const int T = rf_count(A);
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        const int j = next_link(A, T, i);
        if (j >= 0) uf_unite(A.track_id, i, j);
        const int l = leg_link(A, T, i);
        if (l > i) uf_unite(A.track_id, i, l);
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) rf_ids_final(RfArgs A) {
    const int T = rf_count(A);
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        if (A.status[i] != 0) continue;
        // writing a root (an ancestor) keeps every concurrent walk valid
        const int r = uf_root(A.track_id, i);
        __atomic_store_n(A.track_id + i, r, __ATOMIC_RELAXED);
    }
}

// ---------------------------------------------------------------------------
// chain refit

// Measurement of hit k of segment g in its own frame (map-corrected).
__device__ inline void rf_hit(const RfArgs &A, int g, int k, double &x, double &my, double &mz) {
    const int r = A.first_row[g] + k;
    const int c = A.hits[A.offsets[g] + k];
    x = (double)A.row_x[r];
    my = (double)A.y[c];
    mz = (double)A.z[c];
    if (A.map) {
        const float *m = A.map + ((size_t)A.sector[g] * A.n_rows + r) * 2;
        my -= (double)m[0];
        mz -= (double)m[1];
    }
}

__device__ inline bool rf_sane(const RfArgs &A, int g) {
    const int o0 = A.offsets[g], m = A.offsets[g + 1] - o0, r0 = A.first_row[g], s = A.sector[g];
    if (!(m >= 1 && r0 >= 0 && r0 + m <= A.n_rows && s >= 0 && s < A.n_sectors && o0 >= 0 &&
          o0 <= A.cap_hits - m))
        return false;
    for (int k = 0; k < m; ++k)
        if ((uint32_t)A.hits[o0 + k] >= (uint32_t)A.n_clusters) return false;
    return true;
}

// The state p at plane x, rotated into the frame turned by da (cos ca, sin
// sa) and carried along the helix to plane xt there.  J: rows 0..2 of the
// Jacobian (rows 3, 4 are those of the identity): the step's times the
// rotation's, plus the move of the start plane with y.  False if the
// direction leaves the frame's half plane or reaches max_sin.
__device__ inline bool rf_transfer(double p[5], double x, double ca, double sa, double xt, double kbz,
                                   float max_sin, double J[3][5]) {
    const double y = p[0], s = p[2], t = p[3], w = p[4];
    if (!(fabs(s) < 1.0)) return false;
    const double c = sqrt(1.0 - s * s);
    if (!(c * ca + s * sa > 0.0)) return false;
    const double x1 = x * ca + y * sa;
    p[0] = -x * sa + y * ca;
    p[2] = s * ca - c * sa;
    StepJac F;
    if (!helix_step<double, double>(p, xt - x1, kbz, max_sin, F)) return false;
    const double r22 = ca + s / c * sa;
    const double s2 = p[2], c2 = sqrt(1.0 - s2 * s2), kap = kbz * w;
    J[0][0] = ca - sa * s2 / c2; J[0][1] = 0.0; J[0][2] = F.f02 * r22; J[0][3] = 0.0;   J[0][4] = F.f04;
    J[1][0] = -sa * t / c2;      J[1][1] = 1.0; J[1][2] = F.f12 * r22; J[1][3] = F.f13; J[1][4] = F.f14;
    J[2][0] = -sa * kap;         J[2][1] = 0.0; J[2][2] = r22;         J[2][3] = 0.0;   J[2][4] = F.f24;
    return true;
}

__device__ inline void sym_get(const SymT<double> &C, double M[5][5]) {
    M[0][0] = C.c00;
    M[1][0] = M[0][1] = C.c10; M[1][1] = C.c11;
    M[2][0] = M[0][2] = C.c20; M[2][1] = M[1][2] = C.c21; M[2][2] = C.c22;
    M[3][0] = M[0][3] = C.c30; M[3][1] = M[1][3] = C.c31; M[3][2] = M[2][3] = C.c32; M[3][3] = C.c33;
    M[4][0] = M[0][4] = C.c40; M[4][1] = M[1][4] = C.c41; M[4][2] = M[2][4] = C.c42; M[4][3] = M[3][4] = C.c43;
    M[4][4] = C.c44;
}

// C <- J C J^T with rows 3 and 4 of J those of the identity.
__device__ inline void rf_transport(SymT<double> &C, const double J[3][5]) {
    double M[5][5], JC[5][5], R[5][5];
    sym_get(C, M);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            if (i < 3)
                for (int k = 0; k < 5; ++k) acc += J[i][k] * M[k][j];
            else
                acc = M[i][j];
            JC[i][j] = acc;
        }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = 0.0;
            if (j < 3)
                for (int k = 0; k < 5; ++k) acc += JC[i][k] * J[j][k];
            else
                acc = JC[i][j];
            R[i][j] = acc;
        }
    C.c00 = R[0][0];
    C.c10 = R[1][0]; C.c11 = R[1][1];
    C.c20 = R[2][0]; C.c21 = R[2][1]; C.c22 = R[2][2];
    C.c30 = R[3][0]; C.c31 = R[3][1]; C.c32 = R[3][2]; C.c33 = R[3][3];
    C.c40 = R[4][0]; C.c41 = R[4][1]; C.c42 = R[4][2]; C.c43 = R[4][3]; C.c44 = R[4][4];
}

__device__ inline void rf_write(const RfArgs &A, int i, float x, const double p[5], const SymT<double> &C,
                                double chi2, int ndf, int status) {
    A.out.x[i] = x;
    float *po = A.out.par + (size_t)i * 5, *co = A.out.cov + (size_t)i * 15;
    for (int q = 0; q < 5; ++q) po[q] = (float)p[q];
    const double c[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                          C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    for (int q = 0; q < 15; ++q) co[q] = (float)c[q];
    A.out.chi2[i] = (float)chi2;
    A.out.ndf[i] = ndf;
    A.out.status[i] = status;
}

__global__ void __launch_bounds__(TPC_BLOCK) rf_chains(RfArgs A) {
    const int T = rf_count(A);
    for (int h = blockIdx.x * TPC_BLOCK + threadIdx.x; h < T; h += gridDim.x * TPC_BLOCK) {
        double p[5] = {0, 0, 0, 0, 0};
        SymT<double> C = {};
        if (A.status[h] != 0 || prev_link(A, T, h) >= 0) {
            rf_write(A, h, 0.f, p, C, 0.0, 0, TPC_REFIT_NOT_HEAD);
            continue;
        }
        // the chain: length, hits, tail
        int ns = 0, n = 0, tail = h;
        bool sane = true;
        for (int g = h; g >= 0; g = next_link(A, T, g)) {
            if (ns == RF_MAX_CHAIN) {
                ns = -1;
                break;
            }
            ++ns;
            sane = sane && rf_sane(A, g);
            n += A.offsets[g + 1] - A.offsets[g];
            tail = g;
        }
        if (ns < 0) {
            rf_write(A, h, 0.f, p, C, 0.0, 0, TPC_REFIT_LONG_CHAIN);
            continue;
        }
        if (!sane || n < 3) {
            rf_write(A, h, 0.f, p, C, 0.0, 2 * n - 5, TPC_FIT_INIT_FAIL);
            continue;
        }
        // the start: hits 0, (n-1)/2 and n-1, seen from the frame of hit n-1
        const double at = sector_angle(A.sector[tail], A.n_sectors);
        double xa, ya, za, xb, yb, zb, xc, yc, zc;
        const int mt = A.offsets[tail + 1] - A.offsets[tail];
        rf_hit(A, tail, mt - 1, xa, ya, za);
        {
            int g = h, kb = (n - 1) / 2;
            for (;;) {
                const int m = A.offsets[g + 1] - A.offsets[g];
                if (kb < m) break;
                kb -= m;
                g = next_link(A, T, g);
            }
            double x0, y0;
            rf_hit(A, g, kb, x0, y0, zb);
            const double d = sector_angle(A.sector[g], A.n_sectors) - at;
            const double cd = cos(d), sd = sin(d);
            xb = x0 * cd - y0 * sd;
            yb = x0 * sd + y0 * cd;
            rf_hit(A, h, 0, x0, y0, zc);
            const double e = sector_angle(A.sector[h], A.n_sectors) - at;
            const double ce = cos(e), se = sin(e);
            xc = x0 * ce - y0 * se;
            yc = x0 * se + y0 * ce;
        }
        (void)zb;
        int status = TPC_FIT_OK;
        if (!helix_start<double, double>(xa, ya, za, xb, yb, xc, yc, zc, A.kbz, A.max_sin, p))
            status = TPC_FIT_INIT_FAIL;
        C.c00 = A.vy;
        C.c11 = A.vz;
        C.c22 = A.var_s;
        C.c33 = A.var_t;
        C.c44 = A.var_w;
        double chi2 = 0.0, xcur = xa;
        // inwards from the tail's outermost hit
        int g = tail, k = mt - 1;
        while (status == TPC_FIT_OK) {
            double xk, my, mz;
            if (k > 0) {
                --k;
                rf_hit(A, g, k, xk, my, mz);
                StepJac F;
                if (!helix_step<double, double>(p, xk - xcur, A.kbz, A.max_sin, F)) {
                    status = TPC_FIT_SIN_FAIL;
                    break;
                }
                sym_transport<double, false>(C, F);
            } else {
                const int gp = prev_link(A, T, g);
                if (gp < 0) break;
                double da = sector_angle(A.sector[gp], A.n_sectors) - sector_angle(A.sector[g], A.n_sectors);
                const double pi = 3.14159265358979323846;
                if (da > pi) da -= 2.0 * pi;
                if (da < -pi) da += 2.0 * pi;
                g = gp;
                k = A.offsets[g + 1] - A.offsets[g] - 1;
                rf_hit(A, g, k, xk, my, mz);
                double J[3][5];
                if (!rf_transfer(p, xcur, cos(da), sin(da), xk, A.kbz, A.max_sin, J)) {
                    status = TPC_FIT_SIN_FAIL;
                    break;
                }
                rf_transport(C, J);
            }
            xcur = xk;
            const double dchi = kalman_update<double>(p, C, my, mz, A.vy, A.vz);
            chi2 += dchi;
            bool finite = dchi >= 0.0 && isfinite(chi2);
            for (int q = 0; q < 5; ++q) finite = finite && isfinite(p[q]);
            if (!finite) status = TPC_FIT_NUM_FAIL;
        }
        rf_write(A, h, (float)xcur, p, C, chi2, 2 * n - 5, status);
    }
}

// ---------------------------------------------------------------------------
// joint circles of looper legs

__device__ inline int rf_head(const RfArgs &A, int T, int i) {
    for (int step = 0; step < RF_MAX_CHAIN; ++step) {
        const int a = prev_link(A, T, i);
        if (a < 0) return i;
        i = a;
    }
    return -1;
}

// m = (X_c, Y_c, kappa, tan lambda) of the refitted chain at head h and
// S = J C J^T; false for a circle too large or a degenerate state.
__device__ __forceinline__ bool rf_circle(const RfArgs &A, int h, double m[4], double S[4][4]) {
    const float *p = A.out.par + (size_t)h * 5, *co = A.out.cov + (size_t)h * 15;
    const double y = (double)p[0], s = (double)p[2], t = (double)p[3], w = (double)p[4];
    const double k = A.kbz, kap = k * w;
    if (!(fabs(s) < 1.0) || !(fabs(kap) * RF_LEG_MAX_RADIUS > 1.0)) return false;
    const double al = sector_angle(A.sector[h], A.n_sectors);
    const double c = sqrt(1.0 - s * s), ca = cos(al), sa = sin(al);
    const double x = (double)A.out.x[h];
    const double xc = x - s / kap, yc = y + c / kap;
    m[0] = xc * ca - yc * sa;
    m[1] = xc * sa + yc * ca;
    m[2] = kap;
    m[3] = t;
    const double dxc[5] = {0.0, 0.0, -1.0 / kap, 0.0, s * k / (kap * kap)};
    const double dyc[5] = {1.0, 0.0, -s / (c * kap), 0.0, -c * k / (kap * kap)};
    double J[4][5];
    #pragma unroll
    for (int j = 0; j < 5; ++j) {
        J[0][j] = dxc[j] * ca - dyc[j] * sa;
        J[1][j] = dxc[j] * sa + dyc[j] * ca;
        J[2][j] = j == 4 ? k : 0.0;
        J[3][j] = j == 3 ? 1.0 : 0.0;
    }
    double M[5][5];
    #pragma unroll
    for (int a = 0, q = 0; a < 5; ++a)
        #pragma unroll
        for (int b = 0; b <= a; ++b, ++q) M[a][b] = M[b][a] = (double)co[q];
    double JM[4][5];
    #pragma unroll
    for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int b = 0; b < 5; ++b) {
            double acc = 0.0;
            #pragma unroll
            for (int q = 0; q < 5; ++q) acc += J[a][q] * M[q][b];
            JM[a][b] = acc;
        }
    #pragma unroll
    for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int b = 0; b < 4; ++b) {
            double acc = 0.0;
            #pragma unroll
            for (int q = 0; q < 5; ++q) acc += JM[a][q] * J[b][q];
            S[a][b] = acc;
        }
    return true;
}

__global__ void __launch_bounds__(TPC_BLOCK) rf_loops(RfArgs A) {
    const int T = rf_count(A);
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        float *lp = A.loop_par + (size_t)i * 4, *lc = A.loop_cov + (size_t)i * 10;
        #pragma unroll
        for (int q = 0; q < 4; ++q) lp[q] = 0.f;
        #pragma unroll
        for (int q = 0; q < 10; ++q) lc[q] = 0.f;
        A.loop_chi2[i] = -1.f;
        const int j = leg_link(A, T, i);
        if (j <= i) continue;
        const int hi = rf_head(A, T, i), hj = rf_head(A, T, j);
        if (hi < 0 || hj < 0 || hi == hj || A.out.status[hi] != 0 || A.out.status[hj] != 0) continue;
        double mi[4], mj[4], Si[4][4], Sj[4][4];
        if (!rf_circle(A, hi, mi, Si) || !rf_circle(A, hj, mj, Sj)) continue;
        // D S_j D: the (centre, kappa/t) cross terms change sign; S = S_i + D S_j D
        double S[4][4], d[4];
        #pragma unroll
        for (int a = 0; a < 4; ++a)
            #pragma unroll
            for (int b = 0; b < 4; ++b) {
                Sj[a][b] *= ((a < 2) == (b < 2)) ? 1.0 : -1.0;
                S[a][b] = Si[a][b] + Sj[a][b];
            }
        d[0] = mi[0] - mj[0];
        d[1] = mi[1] - mj[1];
        d[2] = mi[2] + mj[2];
        d[3] = mi[3] + mj[3];
        // S = L L^T; chi2 = |L^-1 d|^2
        double L[4][4] = {}, u[4], chi = 0.0;
        bool ok = true;
        #pragma unroll
        for (int a = 0; a < 4 && ok; ++a) {
            #pragma unroll
            for (int b = 0; b <= a; ++b) {
                double acc = S[a][b];
                #pragma unroll
                for (int q = 0; q < b; ++q) acc -= L[a][q] * L[b][q];
                if (a == b) {
                    ok = acc > 0.0;
                    L[a][a] = ok ? sqrt(acc) : 1.0;
                } else {
                    L[a][b] = acc / L[b][b];
                }
            }
            double acc = d[a];
            #pragma unroll
            for (int q = 0; q < a; ++q) acc -= L[a][q] * u[q];
            u[a] = acc / L[a][a];
            chi += u[a] * u[a];
        }
        if (!ok) continue;
        // X = S^-1 S_i (columns by two triangular solves); fused m = m_i - X^T d,
        // C = X^T (D S_j D) symmetrised
        double X[4][4];
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            double v[4];
            #pragma unroll
            for (int a = 0; a < 4; ++a) {
                double acc = Si[a][c];
                #pragma unroll
                for (int q = 0; q < a; ++q) acc -= L[a][q] * v[q];
                v[a] = acc / L[a][a];
            }
            #pragma unroll
            for (int a = 3; a >= 0; --a) {
                double acc = v[a];
                #pragma unroll
                for (int q = a + 1; q < 4; ++q) acc -= L[q][a] * X[q][c];
                X[a][c] = acc / L[a][a];
            }
        }
        #pragma unroll
        for (int a = 0; a < 4; ++a) {
            double acc = mi[a];
            #pragma unroll
            for (int q = 0; q < 4; ++q) acc -= X[q][a] * d[q];
            lp[a] = (float)acc;
        }
        #pragma unroll
        for (int a = 0, q = 0; a < 4; ++a)
            #pragma unroll
            for (int b = 0; b <= a; ++b, ++q) {
                double x1 = 0.0, x2 = 0.0;
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    x1 += X[r][a] * Sj[r][b];
                    x2 += X[r][b] * Sj[r][a];
                }
                lc[q] = (float)(0.5 * (x1 + x2));
            }
        A.loop_chi2[i] = (float)chi;
    }
}

}  // namespace

hipError_t launch_refit(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const tpc_tracks *seg,
                        const int32_t *next, const int32_t *prev, const int32_t *leg, const float *map,
                        int32_t *track_id, const tpc_tracks *out, float *loop_par, float *loop_cov,
                        float *loop_chi2, hipStream_t st) {
    RfArgs A;
    A.offsets = sd->offsets;
    A.hits = sd->hits;
    A.sector = sd->sector;
    A.first_row = sd->first_row;
    A.n_seeds = sd->n_seeds;
    A.cap_seeds = sd->cap_seeds;
    A.cap_hits = sd->cap_hits;
    A.y = fr->y;
    A.z = fr->z;
    A.row_x = ctx->d_row_x;
    A.map = map;
    A.n_rows = ctx->cfg.n_rows;
    A.n_sectors = ctx->cfg.n_sectors;
    A.n_clusters = fr->n_clusters;
    A.kbz = -0.00299792458 * (double)ctx->cfg.bz;
    A.max_sin = ctx->cfg.max_sin;
    A.vy = (double)ctx->cfg.sigma_y * (double)ctx->cfg.sigma_y;
    A.vz = (double)ctx->cfg.sigma_z * (double)ctx->cfg.sigma_z;
    A.var_s = (double)ctx->cfg.var_sin0;
    A.var_t = (double)ctx->cfg.var_tgl0;
    A.var_w = (double)ctx->cfg.var_qpt0;
    A.status = seg->status;
    A.next = next;
    A.prev = prev;
    A.leg = leg;
    A.track_id = track_id;
    A.out = *out;
    A.loop_par = loop_par;
    A.loop_cov = loop_cov;
    A.loop_chi2 = loop_chi2;
    int g = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(rf_ids_init, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(rf_ids_union, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(rf_ids_final, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(rf_chains, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    if (loop_par) hipLaunchKernelGGL(rf_loops, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}
