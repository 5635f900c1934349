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

// Candidates of one lane that pass the tan(lambda) / q/pT test, per chunk of
// the neighbouring sector's segments: kept in the lane's own LDS column, so
// that the transfer runs over short lists (a wavefront's iterations are the
// longest list of its lanes) instead of every candidate of every lane.
#define MG_CHUNK 64

__global__ void __launch_bounds__(TPC_BLOCK) mg_best(MgArgs A) {
    __shared__ int cand[MG_CHUNK][TPC_BLOCK];
    const int T = mg_count(A);
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK) {
        int bo = -1, bi = -1;
        double co = INFINITY, ci_ = INFINITY;
        if (A.status[i] == 0 && A.n_sectors == 36) {
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
                    for (int j = c0; j < c1; ++j) {
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
        A.next[i] = bo;
        A.chi2[i] = bo >= 0 ? (float)co : 0.f;
        A.prev[i] = bi;
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
    double S[4][4];       // J C J^T
};

// The circle of segment i (false if too large or degenerate).
__device__ bool leg_circle(const MgArgs &A, int i, Circle &o) {
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
    for (int j = 0; j < 5; ++j) {
        J[0][j] = dxc[j] * ca - dyc[j] * sa;
        J[1][j] = dxc[j] * sa + dyc[j] * ca;
        J[2][j] = j == 4 ? k : 0.0;
        J[3][j] = j == 3 ? 1.0 : 0.0;
    }
    double C[5][5];
    for (int a = 0, q = 0; a < 5; ++a)
        for (int b = 0; b <= a; ++b, ++q) C[a][b] = C[b][a] = (double)co[q];
    double JC[4][5];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 5; ++b) {
            double acc = 0.0;
            for (int q = 0; q < 5; ++q) acc += J[a][q] * C[q][b];
            JC[a][b] = acc;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double acc = 0.0;
            for (int q = 0; q < 5; ++q) acc += JC[a][q] * J[b][q];
            o.S[a][b] = acc;
        }
    return true;
}

__global__ void __launch_bounds__(TPC_BLOCK) lg_best(MgArgs A) {
    __shared__ int cand[MG_CHUNK][TPC_BLOCK];
    const int T = mg_count(A);
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const double k2 = A.kbz * A.kbz;
    // whole workgroups step together, so every lane of a wavefront stays in
    // the loop body (the shuffles below need them all)
    for (int base = blockIdx.x * TPC_BLOCK; base < T; base += gridDim.x * TPC_BLOCK) {
        const int i = base + threadIdx.x;
        int best = -1;
        double bchi = INFINITY;
        Circle ci;
        const bool live = i < T && A.status[i] == 0 && A.n_sectors == 36 && leg_circle(A, i, ci);
        int j0 = 0, j1 = 0;
        double wi = 0.0, ti = 0.0, vwi = 0.0, vti = 0.0;
        if (live) {
            const int64_t key = (int64_t)A.frame[i] * A.n_sectors + (A.sector[i] / 18) * 18;
            j0 = mg_lower(A, T, key);
            j1 = mg_lower(A, T, key + 18);
            wi = (double)A.par[(size_t)i * 5 + 4];
            ti = (double)A.par[(size_t)i * 5 + 3];
            vwi = (double)A.cov[(size_t)i * 15 + 14];
            vti = (double)A.cov[(size_t)i * 15 + 9];
        }
        // one candidate range for every live lane (its segments share a frame
        // and side): lanes load one candidate each per chunk and test it on
        // shuffled copies; otherwise each lane walks its own range
        const unsigned long long lv = __ballot(live);
        const int lead = lv ? __ffsll((long long)lv) - 1 : 0;
        const int L0 = __shfl(j0, lead), L1 = __shfl(j1, lead);
        const bool shared_range = __all(!live || (j0 == L0 && j1 == L1));
        const int r0 = shared_range ? L0 : j0, r1 = shared_range ? L1 : j1;
        for (int c0 = r0; c0 < r1; c0 += MG_CHUNK) {
            const int c1 = c0 + MG_CHUNK < r1 ? c0 + MG_CHUNK : r1;
            int n = 0;
            if (shared_range) {
                const int jl = c0 + lane;
                double wq = 0.0, tq = 0.0, vwq = 0.0, vtq = 0.0;
                int okq = 0;
                if (jl < c1) {
                    okq = A.status[jl] == 0;
                    wq = (double)A.par[(size_t)jl * 5 + 4];
                    tq = (double)A.par[(size_t)jl * 5 + 3];
                    vwq = (double)A.cov[(size_t)jl * 15 + 14];
                    vtq = (double)A.cov[(size_t)jl * 15 + 9];
                }
                for (int q = 0; q < c1 - c0; ++q) {
                    const int ok = __shfl(okq, q);
                    const double wj = __shfl(wq, q), tj = __shfl(tq, q);
                    const double vwj = __shfl(vwq, q), vtj = __shfl(vtq, q);
                    const double dk = A.kbz * (wi + wj), dt = ti + tj;
                    if (live && ok && c0 + q != i && !(dk * dk > A.cut * k2 * (vwi + vwj)) &&
                        !(dt * dt > A.cut * (vti + vtj)))
                        cand[n++][threadIdx.x] = c0 + q;
                }
            } else if (live) {
                for (int j = c0; j < c1; ++j) {
                    if (j == i || A.status[j] != 0) continue;
                    const float *pj = A.par + (size_t)j * 5, *cj = A.cov + (size_t)j * 15;
                    // curvature and tan(lambda) alone (their rows of J are exact
                    // and need no circle): a pair failing either cannot pass
                    const double dk = A.kbz * (wi + (double)pj[4]), dt = ti + (double)pj[3];
                    if (dk * dk > A.cut * k2 * (vwi + (double)cj[14]) || dt * dt > A.cut * (vti + (double)cj[9]))
                        continue;
                    cand[n++][threadIdx.x] = j;
                }
            }
            for (int q = 0; q < n; ++q) {
                const int j = cand[q][threadIdx.x];
                Circle cj;
                if (!leg_circle(A, j, cj)) continue;
                double S[4][4], d[4];
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b)
                        S[a][b] = ci.S[a][b] + (((a < 2) == (b < 2)) ? 1.0 : -1.0) * cj.S[a][b];
                d[0] = ci.m[0] - cj.m[0];
                d[1] = ci.m[1] - cj.m[1];
                d[2] = ci.m[2] + cj.m[2];
                d[3] = ci.m[3] + cj.m[3];
                // chi2 = |L^-1 d|^2, S = L L^T
                double L[4][4], z[4], chi = 0.0;
                bool ok = true;
                for (int a = 0; a < 4 && ok; ++a) {
                    for (int b = 0; b <= a; ++b) {
                        double acc = S[a][b];
                        for (int m = 0; m < b; ++m) acc -= L[a][m] * L[b][m];
                        if (a == b) {
                            if (!(acc > 0.0)) { ok = false; break; }
                            L[a][a] = sqrt(acc);
                        } else {
                            L[a][b] = acc / L[b][b];
                        }
                    }
                    if (!ok) break;
                    double acc = d[a];
                    for (int m = 0; m < a; ++m) acc -= L[a][m] * z[m];
                    z[a] = acc / L[a][a];
                    chi += z[a] * z[a];
                }
                if (ok && chi > 0.0 && chi <= A.cut && (chi < bchi || (chi == bchi && j < best))) {
                    bchi = chi;
                    best = j;
                }
            }
        }
        if (i < T) {
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
    hipLaunchKernelGGL(mg_best, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(mg_link_next, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(mg_link_prev, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    if (leg) {
        hipLaunchKernelGGL(lg_best, dim3(g), dim3(TPC_BLOCK), 0, st, A);
        hipLaunchKernelGGL(lg_link, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    }
    return hipGetLastError();
}
