// Merging of fitted track segments across sector edges (gfx950).  A particle
// that crosses from one sector into the next on the same side leaves a
// fitted segment in each; carried to a common plane, their states agree
// within their covariances.
//
//  mg_best         thread per segment: over the segments of the two
//                  neighbouring sectors of its (frame, side) -- a contiguous
//                  seed range each, found by binary search, since seeds are
//                  ordered by first cluster and clusters by (frame, sector,
//                  row) -- its best outer partner (its innermost point at
//                  the smaller radius) and best inner partner: smallest chi2
//                  <= cut, smaller index on ties.  Pairs whose (tan(lambda),
//                  q/pT) difference alone has a chi2 above the cut are
//                  dropped first (both are unchanged by the transfer, so
//                  their covariance block is the sum of the two segments',
//                  and a sub-vector's chi2 never exceeds the full one: such a
//                  pair cannot pass); the survivors of each chunk of
//                  64 candidates go to the lane's own LDS column and only
//                  they are transferred.  FP64 throughout.
//  mg_link_next    next[a] = b when a's best outer partner b has a as its
//                  best inner partner (else -1, chi2 0); optionally the pair
//                  combined at b's plane (a's transferred state fused with
//                  b's: the joint fit of both for the linearised problem)
//  mg_link_prev    prev[b] = a when next[a] = b
//  lg_best, lg_link  optionally, the legs of loopers: per segment the
//                  best partner among the segments of its frame and side
//                  whose circle matches with curvature and tan(lambda)
//                  reversed, then mutual best
//
// The transfer: a state at plane x of the inner segment's frame is rotated
// into the outer segment's frame (turned by da: a point (x, y) ->
// (x cos da + y sin da, -x sin da + y cos da), phi -> phi - da, cos phi > 0
// kept) and carried along the helix to the outer segment's innermost plane;
// its Jacobian is the step's (at fixed distance) times the rotation's, plus
// the move of the start plane with y, which shortens the step.
#include "tpc_fit_math.hpp"
#include "tpc_merge.hpp"

namespace {

struct MgArgs {
    const float *x, *par, *cov;
    const int32_t *status, *frame, *sector, *n_seeds;
    int32_t cap, n_sectors;
    double kbz, cut;
    float max_sin;
    int32_t *next, *prev;
    float *chi2;
    float *mpar, *mcov;      // optional combined states of linked pairs
    int32_t *leg;            // optional pairing of the legs of loopers
    float *leg_chi2;
};

__device__ inline int mg_count(const MgArgs &A) {
    const int n = *A.n_seeds;
    return n < 0 ? 0 : (n < A.cap ? n : A.cap);
}

__device__ inline int64_t mg_key(const MgArgs &A, int i) {
    return (int64_t)A.frame[i] * A.n_sectors + A.sector[i];
}

// First seed index in [0, T) whose key is >= k.
__device__ inline int mg_lower(const MgArgs &A, int T, int64_t k) {
    int lo = 0, hi = T;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (mg_key(A, mid) < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ inline double sector_angle(int sec, int n_sectors) {
    const double pi = 3.14159265358979323846;
    return n_sectors == 1 ? 0.0 : (double)(sec % 18) * (pi / 9.0) + pi / 18.0;
}

// The angle that turns sector a's frame into sector b's, wrapped to (-pi, pi].
__device__ inline double turn_angle(int sa, int sb, int n_sectors) {
    const double pi = 3.14159265358979323846;
    double da = sector_angle(sb, n_sectors) - sector_angle(sa, n_sectors);
    if (da > pi) da -= 2.0 * pi;
    if (da < -pi) da += 2.0 * pi;
    return da;
}

// chi2 of carrying segment a onto segment b (INFINITY if it cannot be
// formed); ca, sa: cos and sin of the turn from a's sector to b's.  With mp,
// mc non-null also the two combined at b's plane: a's transferred state
// (covariance P = J C_a J^T) and b's fused, x = p_a' + P S^-1 (p_b - p_a'),
// C = P S^-1 C_b (= P - P S^-1 P), S = P + C_b (packed, in float).
__device__ double pair_fuse(const MgArgs &A, int a, int b, double ca, double sa, float *mp, float *mc) {
    const float *pa = A.par + (size_t)a * 5, *pb = A.par + (size_t)b * 5;
    const double x = (double)A.x[a], y = (double)pa[0], s = (double)pa[2], t = (double)pa[3], w = (double)pa[4];
    if (!(fabs(s) < 1.0)) return INFINITY;
    const double c = sqrt(1.0 - s * s);
    if (!(c * ca + s * sa > 0.0)) return INFINITY;
    const double x1 = x * ca + y * sa;
    double q[5] = {-x * sa + y * ca, (double)pa[1], s * ca - c * sa, t, w};
    StepJac F;
    if (!helix_step<double, double>(q, (double)A.x[b] - x1, A.kbz, A.max_sin, F)) return INFINITY;
    // J = F R - v e_0^T sin(da), R = diag(ca, 1, ca + (s/c) sa, 1, 1), v = (s2/c2, t/c2, kappa, 0, 0)
    const double r22 = ca + s / c * sa;
    const double s2 = q[2], c2 = sqrt(1.0 - s2 * s2), kap = A.kbz * w;
    double J[3][5];
    J[0][0] = ca - sa * s2 / c2; J[0][1] = 0.0; J[0][2] = F.f02 * r22; J[0][3] = 0.0;   J[0][4] = F.f04;
    J[1][0] = -sa * t / c2;      J[1][1] = 1.0; J[1][2] = F.f12 * r22; J[1][3] = F.f13; J[1][4] = F.f14;
    J[2][0] = -sa * kap;         J[2][1] = 0.0; J[2][2] = r22;         J[2][3] = 0.0;   J[2][4] = F.f24;
    double Ca[5][5], Cb[5][5], S[5][5], P[5][5];
    const float *ca_ = A.cov + (size_t)a * 15, *cb_ = A.cov + (size_t)b * 15;
    for (int i = 0, k = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j, ++k) {
            Ca[i][j] = Ca[j][i] = (double)ca_[k];
            S[i][j] = S[j][i] = Cb[i][j] = Cb[j][i] = (double)cb_[k];
        }
    // S += J Ca J^T, with rows 3 and 4 of J those of the identity
    double JC[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            if (i < 3)
                for (int k = 0; k < 5; ++k) acc += J[i][k] * Ca[k][j];
            else
                acc = Ca[i][j];
            JC[i][j] = acc;
        }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            double acc = 0.0;
            if (j < 3)
                for (int k = 0; k < 5; ++k) acc += JC[i][k] * J[j][k];
            else
                acc = JC[i][j];
            P[i][j] = P[j][i] = acc;
            S[i][j] += acc;
            if (j != i) S[j][i] = S[i][j];
        }
    double d[5];
    for (int i = 0; i < 5; ++i) d[i] = q[i] - (double)pb[i];
    // chi2 = |L^-1 d|^2 with S = L L^T
    double L[5][5], z[5], chi = 0.0;
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j <= i; ++j) {
            double acc = S[i][j];
            for (int k = 0; k < j; ++k) acc -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(acc > 0.0)) return INFINITY;
                L[i][i] = sqrt(acc);
            } else {
                L[i][j] = acc / L[j][j];
            }
        }
        double acc = d[i];
        for (int k = 0; k < i; ++k) acc -= L[i][k] * z[k];
        z[i] = acc / L[i][i];
        chi += z[i] * z[i];
    }
    if (mp && mc) {
        // X = S^-1 P by the two triangular solves, column by column
        double X[5][5];
        for (int c = 0; c < 5; ++c) {
            double y[5];
            for (int i = 0; i < 5; ++i) {
                double acc = P[i][c];
                for (int k = 0; k < i; ++k) acc -= L[i][k] * y[k];
                y[i] = acc / L[i][i];
            }
            for (int i = 4; i >= 0; --i) {
                double acc = y[i];
                for (int k = i + 1; k < 5; ++k) acc -= L[k][i] * X[k][c];
                X[i][c] = acc / L[i][i];
            }
        }
        // d = p_a' - p_b: x = p_a' - P S^-1 d = p_a' - X^T d
        for (int i = 0; i < 5; ++i) {
            double acc = q[i];
            for (int k = 0; k < 5; ++k) acc -= X[k][i] * d[k];
            mp[i] = (float)acc;
        }
        // C = P S^-1 C_b = X^T C_b, symmetrised (equal to P - P S^-1 P, with
        // no difference of large terms when one covariance dwarfs the other)
        for (int i = 0, k = 0; i < 5; ++i)
            for (int j = 0; j <= i; ++j, ++k) {
                double u = 0.0, v = 0.0;
                for (int m = 0; m < 5; ++m) {
                    u += X[m][i] * Cb[m][j];
                    v += X[m][j] * Cb[m][i];
                }
                mc[k] = (float)(0.5 * (u + v));
            }
    }
    return chi > 0.0 ? chi : INFINITY;
}

__device__ inline double pair_chi2(const MgArgs &A, int a, int b, double ca, double sa) {
    return pair_fuse(A, a, b, ca, sa, nullptr, nullptr);
}

// MG_SPLIT lanes of one wavefront share a segment and take every
// MG_SPLIT-th candidate of each neighbouring sector (enough wavefronts for
// the chip); their best partners are reduced by shuffles at the end
// (smaller chi2, then smaller index: the serial order's choice).  Per chunk
// of MG_CHUNK candidates, the ones that pass the tan(lambda) / q/pT test go
// to the lane's own LDS column, so that the transfer runs over short lists
// (a wavefront's iterations are the longest list of its lanes) instead of
// every candidate of every lane.
#define MG_SPLIT 4
#define MG_CHUNK 64
#define MG_LANE_CHUNK (MG_CHUNK / MG_SPLIT)

// (chi, j) of another lane replaces this lane's best when smaller, or equal
// with a smaller index
__device__ inline void best_merge(double &chi, int &j, double oc, int oj) {
    if (oc < chi || (oc == chi && oj >= 0 && (j < 0 || oj < j))) {
        chi = oc;
        j = oj;
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) mg_best(MgArgs A) {
    __shared__ int cand[MG_LANE_CHUNK][TPC_BLOCK];
    const int T = mg_count(A);
    const int sub = threadIdx.x % MG_SPLIT;
    const int per_block = TPC_BLOCK / MG_SPLIT;
    // whole workgroups step together: every lane reaches the shuffles
    for (int base = blockIdx.x * per_block; base < T; base += gridDim.x * per_block) {
        const int i = base + threadIdx.x / MG_SPLIT;
        int bo = -1, bi = -1;
        double co = INFINITY, ci_ = INFINITY;
        if (i < T && A.status[i] == 0 && A.n_sectors == 36) {
            const float *pi_ = A.par + (size_t)i * 5, *ci = A.cov + (size_t)i * 15;
            const double ri = hypot((double)A.x[i], (double)pi_[0]);
            const double ti = (double)pi_[3], wi = (double)pi_[4], vti = (double)ci[9], vwi = (double)ci[14];
            const double cti = (double)ci[13];
            const int sec = A.sector[i], side = sec / 18, s18 = sec % 18;
            for (int e = 0; e < 2; ++e) {
                const int sn = side * 18 + (e == 0 ? (s18 + 1) % 18 : (s18 + 17) % 18);
                const int64_t key = (int64_t)A.frame[i] * A.n_sectors + sn;
                const int j0 = mg_lower(A, T, key), j1 = mg_lower(A, T, key + 1);
                // the turn from this sector to the neighbour's (outer partners) and back
                const double da = turn_angle(sec, sn, A.n_sectors);
                const double cda = cos(da), sda = sin(da);
                const double dback = turn_angle(sn, sec, A.n_sectors);
                const double cdb = cos(dback), sdb = sin(dback);
                for (int c0 = j0; c0 < j1; c0 += MG_CHUNK) {
                    const int c1 = c0 + MG_CHUNK < j1 ? c0 + MG_CHUNK : j1;
                    int n = 0;
                    for (int j = c0 + sub; j < c1; j += MG_SPLIT) {
                        if (A.status[j] != 0) continue;
                        const float *pj = A.par + (size_t)j * 5, *cj = A.cov + (size_t)j * 15;
                        // the (t, w) block of the pair's covariance is the sum of the
                        // two (the transfer leaves t and w alone), and its chi2
                        // never exceeds the full one
                        const double dt = ti - (double)pj[3], dw = wi - (double)pj[4];
                        const double s33 = vti + (double)cj[9], s44 = vwi + (double)cj[14];
                        const double s43 = cti + (double)cj[13];
                        const double det = s33 * s44 - s43 * s43;
                        if (det > 0.0 && (s44 * dt * dt - 2.0 * s43 * dt * dw + s33 * dw * dw) > A.cut * det)
                            continue;
                        cand[n++][threadIdx.x] = j;
                    }
                    for (int k = 0; k < n; ++k) {
                        const int j = cand[k][threadIdx.x];
                        const double rj = hypot((double)A.x[j], (double)A.par[(size_t)j * 5]);
                        if (ri < rj) {                        // j outside: an outer partner
                            const double chi = pair_chi2(A, i, j, cda, sda);
                            if (chi <= A.cut && (chi < co || (chi == co && j < bo))) {
                                co = chi;
                                bo = j;
                            }
                        } else if (rj < ri) {                 // an inner partner
                            const double chi = pair_chi2(A, j, i, cdb, sdb);
                            if (chi <= A.cut && (chi < ci_ || (chi == ci_ && j < bi))) {
                                ci_ = chi;
                                bi = j;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int d = 1; d < MG_SPLIT; d <<= 1) {
            best_merge(co, bo, __shfl_xor(co, d, TPC_WAVE), __shfl_xor(bo, d, TPC_WAVE));
            best_merge(ci_, bi, __shfl_xor(ci_, d, TPC_WAVE), __shfl_xor(bi, d, TPC_WAVE));
        }
        if (i < T && sub == 0) {
            A.next[i] = bo;
            A.chi2[i] = bo >= 0 ? (float)co : 0.f;
            A.prev[i] = bi;
        }
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) mg_link_next(MgArgs A) {
    const int T = mg_count(A);
    for (int a = blockIdx.x * TPC_BLOCK + threadIdx.x; a < T; a += gridDim.x * TPC_BLOCK) {
        const int b = A.next[a];
        const bool linked = b >= 0 && b < T && A.prev[b] == a;
        if (!linked) {
            A.next[a] = -1;
            A.chi2[a] = 0.f;
        }
        if (A.mpar) {
            float *mp = A.mpar + (size_t)a * 5, *mc = A.mcov + (size_t)a * 15;
            for (int q = 0; q < 5; ++q) mp[q] = 0.f;
            for (int q = 0; q < 15; ++q) mc[q] = 0.f;
            if (linked) {
                const double da = turn_angle(A.sector[a], A.sector[b], A.n_sectors);
                pair_fuse(A, a, b, cos(da), sin(da), mp, mc);
            }
        }
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) mg_link_prev(MgArgs A) {
    const int T = mg_count(A);
    for (int b = blockIdx.x * TPC_BLOCK + threadIdx.x; b < T; b += gridDim.x * TPC_BLOCK) {
        const int a = A.prev[b];
        if (!(a >= 0 && a < T && A.next[a] == b)) A.prev[b] = -1;
    }
}

// ---------------------------------------------------------------------------
// Legs of loopers.  A returning leg is fitted as a track running outwards
// along the same circle in the other sense: the same centre, curvature and
// tan(lambda) of opposite signs.  m = (X_c, Y_c, kappa, t) per segment in
// global coordinates, compared as m_A - D m_B, D = diag(1, 1, -1, -1), with
// chi2 = d^T (J_A C_A J_A^T + D J_B C_B J_B^T D)^-1 d (4 dof).  Candidates:
// fitted segments of one frame and side in any sectors, circle radius below
// 250 cm.

#define LEG_MAX_RADIUS 250.0

struct Circle {
    double m[4];
    double s00, s10, s11, s20, s21, s22, s30, s31, s32, s33;   // J C J^T, lower triangle
};

// The circle of segment i (false if too large or degenerate).
__device__ __forceinline__ bool leg_circle(const MgArgs &A, int i, Circle &o) {
    const float *p = A.par + (size_t)i * 5, *co = A.cov + (size_t)i * 15;
    const double y = (double)p[0], s = (double)p[2], t = (double)p[3], w = (double)p[4];
    const double k = A.kbz, kap = k * w;
    if (!(fabs(s) < 1.0) || !(fabs(kap) * LEG_MAX_RADIUS > 1.0)) return false;
    const double al = sector_angle(A.sector[i], A.n_sectors);
    const double c = sqrt(1.0 - s * s), ca = cos(al), sa = sin(al);
    const double x = (double)A.x[i];
    const double xc = x - s / kap, yc = y + c / kap;
    o.m[0] = xc * ca - yc * sa;
    o.m[1] = xc * sa + yc * ca;
    o.m[2] = kap;
    o.m[3] = t;
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
    double C[5][5];
#pragma unroll
    for (int a = 0, q = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b, ++q) C[a][b] = C[b][a] = (double)co[q];
    double JC[4][5];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) acc += J[a][q] * C[q][b];
            JC[a][b] = acc;
        }
    double S[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) acc += JC[a][q] * J[b][q];
            S[a][b] = acc;
        }
    o.s00 = S[0][0];
    o.s10 = S[1][0]; o.s11 = S[1][1];
    o.s20 = S[2][0]; o.s21 = S[2][1]; o.s22 = S[2][2];
    o.s30 = S[3][0]; o.s31 = S[3][1]; o.s32 = S[3][2]; o.s33 = S[3][3];
    return true;
}

// chi2 of legs a and b (m_a - D m_b against S_a + D S_b D, D = diag(1, 1,
// -1, -1): the (centre, kappa/t) cross terms of S_b change sign), by a 4x4
// Cholesky; INFINITY if the sum is not positive definite.
__device__ __forceinline__ double leg_chi2(const Circle &a, const Circle &b) {
    const double d0 = a.m[0] - b.m[0], d1 = a.m[1] - b.m[1], d2 = a.m[2] + b.m[2], d3 = a.m[3] + b.m[3];
    const double S00 = a.s00 + b.s00, S10 = a.s10 + b.s10, S11 = a.s11 + b.s11;
    const double S20 = a.s20 - b.s20, S21 = a.s21 - b.s21, S22 = a.s22 + b.s22;
    const double S30 = a.s30 - b.s30, S31 = a.s31 - b.s31, S32 = a.s32 + b.s32, S33 = a.s33 + b.s33;
    bool ok = S00 > 0.0;
    const double L00 = sqrt(ok ? S00 : 1.0);
    const double L10 = S10 / L00, L20 = S20 / L00, L30 = S30 / L00;
    const double e11 = S11 - L10 * L10;
    ok = ok && e11 > 0.0;
    const double L11 = sqrt(ok ? e11 : 1.0);
    const double L21 = (S21 - L20 * L10) / L11, L31 = (S31 - L30 * L10) / L11;
    const double e22 = S22 - L20 * L20 - L21 * L21;
    ok = ok && e22 > 0.0;
    const double L22 = sqrt(ok ? e22 : 1.0);
    const double L32 = (S32 - L30 * L20 - L31 * L21) / L22;
    const double e33 = S33 - L30 * L30 - L31 * L31 - L32 * L32;
    ok = ok && e33 > 0.0;
    const double L33 = sqrt(ok ? e33 : 1.0);
    const double z0 = d0 / L00;
    const double z1 = (d1 - L10 * z0) / L11;
    const double z2 = (d2 - L20 * z0 - L21 * z1) / L22;
    const double z3 = (d3 - L30 * z0 - L31 * z1 - L32 * z2) / L33;
    return ok ? z0 * z0 + z1 * z1 + z2 * z2 + z3 * z3 : INFINITY;
}

// Candidates are the segments of the segment's (frame, side): one
// contiguous seed range.  LG_SPLIT lanes of one wavefront share a segment
// and take every LG_SPLIT-th candidate, so that the chip holds enough
// wavefronts; their best candidates are reduced by shuffles at the end
// (smaller chi2, then smaller index: the serial order's choice).  The
// workgroup walks the union of its segments' ranges in tiles of TPC_BLOCK
// segments: each thread forms the circle of one tile segment into LDS, then
// the lanes test the tile from there.  Each circle is formed once per
// workgroup and tile instead of once per pair.
#define LG_SPLIT 8
#define LG_SEGS (TPC_BLOCK / LG_SPLIT)

struct LegTile {
    double m[4][TPC_BLOCK];
    double s[10][TPC_BLOCK];
    int ok[TPC_BLOCK];
};

__global__ void __launch_bounds__(TPC_BLOCK) lg_best(MgArgs A) {
    __shared__ LegTile tile;
    __shared__ int span[2];
    const int T = mg_count(A);
    const int sub = threadIdx.x % LG_SPLIT;
    // whole workgroups step together: every lane reaches the barriers and
    // the shuffles
    for (int base = blockIdx.x * LG_SEGS; base < T; base += gridDim.x * LG_SEGS) {
        const int i = base + threadIdx.x / LG_SPLIT;
        int best = -1;
        double bchi = INFINITY;
        Circle ci;
        const bool live = i < T && A.status[i] == 0 && A.n_sectors == 36 && leg_circle(A, i, ci);
        int j0 = T, j1 = 0;
        if (live) {
            const int64_t key = (int64_t)A.frame[i] * A.n_sectors + (A.sector[i] / 18) * 18;
            j0 = mg_lower(A, T, key);
            j1 = mg_lower(A, T, key + 18);
        }
        if (threadIdx.x == 0) {
            span[0] = T;
            span[1] = 0;
        }
        __syncthreads();
        if (live && sub == 0) {
            atomicMin(&span[0], j0);
            atomicMax(&span[1], j1);
        }
        __syncthreads();
        const int u0 = span[0], u1 = span[1];
        for (int c0 = u0; c0 < u1; c0 += TPC_BLOCK) {
            const int c = c0 + threadIdx.x;
            Circle cc;
            const bool okc = c < u1 && A.status[c] == 0 && leg_circle(A, c, cc);
            tile.ok[threadIdx.x] = okc;
            if (okc) {
#pragma unroll
                for (int q = 0; q < 4; ++q) tile.m[q][threadIdx.x] = cc.m[q];
                tile.s[0][threadIdx.x] = cc.s00; tile.s[1][threadIdx.x] = cc.s10; tile.s[2][threadIdx.x] = cc.s11;
                tile.s[3][threadIdx.x] = cc.s20; tile.s[4][threadIdx.x] = cc.s21; tile.s[5][threadIdx.x] = cc.s22;
                tile.s[6][threadIdx.x] = cc.s30; tile.s[7][threadIdx.x] = cc.s31; tile.s[8][threadIdx.x] = cc.s32;
                tile.s[9][threadIdx.x] = cc.s33;
            }
            __syncthreads();
            const int n = u1 - c0 < TPC_BLOCK ? u1 - c0 : TPC_BLOCK;
            if (live) {
                const int q0 = j0 > c0 ? j0 - c0 : 0;
                const int q1 = j1 - c0 < n ? j1 - c0 : n;
                // this lane's candidates: q = sub (mod LG_SPLIT) in [q0, q1)
                for (int q = q0 + ((sub - q0 % LG_SPLIT + LG_SPLIT) % LG_SPLIT); q < q1; q += LG_SPLIT) {
                    const int j = c0 + q;
                    if (!tile.ok[q] || j == i) continue;
                    // curvature and tan(lambda) alone (exact rows of J): a pair
                    // failing either cannot pass the full test
                    const double dk = ci.m[2] + tile.m[2][q], dt = ci.m[3] + tile.m[3][q];
                    if (dk * dk > A.cut * (ci.s22 + tile.s[5][q]) || dt * dt > A.cut * (ci.s33 + tile.s[9][q]))
                        continue;
                    Circle cj;
                    cj.m[0] = tile.m[0][q]; cj.m[1] = tile.m[1][q]; cj.m[2] = tile.m[2][q]; cj.m[3] = tile.m[3][q];
                    cj.s00 = tile.s[0][q]; cj.s10 = tile.s[1][q]; cj.s11 = tile.s[2][q]; cj.s20 = tile.s[3][q];
                    cj.s21 = tile.s[4][q]; cj.s22 = tile.s[5][q]; cj.s30 = tile.s[6][q]; cj.s31 = tile.s[7][q];
                    cj.s32 = tile.s[8][q]; cj.s33 = tile.s[9][q];
                    const double chi = leg_chi2(ci, cj);
                    if (chi > 0.0 && chi <= A.cut && chi < bchi) {   // j ascends: ties keep the smaller
                        bchi = chi;
                        best = j;
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int d = 1; d < LG_SPLIT; d <<= 1) {
            best_merge(bchi, best, __shfl_xor(bchi, d, TPC_WAVE), __shfl_xor(best, d, TPC_WAVE));
        }
        if (i < T && sub == 0) {
            A.leg[i] = best;
            A.leg_chi2[i] = best >= 0 ? (float)bchi : 0.f;
        }
    }
}

// Mutual best, in place: a segment whose best does not choose it back is
// cleared; the value another thread reads can only change from "not me" to
// -1, and a mutual pair is never cleared.
__global__ void __launch_bounds__(TPC_BLOCK) lg_link(MgArgs A) {
    const int T = mg_count(A);
    for (int a = blockIdx.x * TPC_BLOCK + threadIdx.x; a < T; a += gridDim.x * TPC_BLOCK) {
        const int b = A.leg[a];
        if (!(b >= 0 && b < T && A.leg[b] == a)) {
            A.leg[a] = -1;
            A.leg_chi2[a] = 0.f;
        }
    }
}

}  // namespace

hipError_t launch_merge(const tpc_context *ctx, const tpc_seeds *sd, const tpc_tracks *tr, double cut,
                        int32_t *next, int32_t *prev, float *chi2, float *mpar, float *mcov, int32_t *leg,
                        float *leg_chi2, hipStream_t st) {
    MgArgs A;
    A.x = tr->x;
    A.par = tr->par;
    A.cov = tr->cov;
    A.status = tr->status;
    A.frame = sd->frame;
    A.sector = sd->sector;
    A.n_seeds = sd->n_seeds;
    A.cap = sd->cap_seeds;
    A.n_sectors = ctx->cfg.n_sectors;
    A.kbz = -0.00299792458 * (double)ctx->cfg.bz;
    A.cut = cut;
    A.max_sin = ctx->cfg.max_sin;
    A.next = next;
    A.prev = prev;
    A.chi2 = chi2;
    A.mpar = mpar;
    A.mcov = mcov;
    A.leg = leg;
    A.leg_chi2 = leg_chi2;
    int g = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    int gm = (int)(((int64_t)sd->cap_seeds * MG_SPLIT + TPC_BLOCK - 1) / TPC_BLOCK);
    gm = gm < 1 ? 1 : (gm > 8192 ? 8192 : gm);
    hipLaunchKernelGGL(mg_best, dim3(gm), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(mg_link_next, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(mg_link_prev, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    if (leg) {
        int gl = (int)(((int64_t)sd->cap_seeds * LG_SPLIT + TPC_BLOCK - 1) / TPC_BLOCK);
        gl = gl < 1 ? 1 : (gl > 8192 ? 8192 : gl);
        hipLaunchKernelGGL(lg_best, dim3(gl), dim3(TPC_BLOCK), 0, st, A);
        hipLaunchKernelGGL(lg_link, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    }
    return hipGetLastError();
}
