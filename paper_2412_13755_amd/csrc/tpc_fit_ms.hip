// Kalman fit with material (gfx950): the seed fit with multiple scattering
// in the gas as process noise and rejection of outlying hits; the same
// kernel also fits seeds whose hits skip pad rows, with per-cluster errors.
//
//  fit_ms_tracks  thread per seed, double precision (plane distances and
//                 -c Bz too): three-point start at the outermost hit; for
//                 each inward step, the scattering of the segment about to
//                 be crossed enters the covariance (Highland, from the state
//                 at the plane the step leaves), then the helix step and
//                 transport (with energy loss, the loss of the segment
//                 is given back between the two, a map of q/pT whose
//                 Jacobian and straggling noise enter the covariance);
//                 the hit's predicted-residual chi2 decides
//                 whether it is used (update) or rejected (flagged).  The
//                 next hit's coordinates are loaded a step ahead.
//                 ROWS: the pad row of every hit is looked up in the
//                 cluster layout of the seed's (frame, sector) -- a binary
//                 search for the outermost hit, then a walk down from the
//                 row above for each next one (at most R + n reads of the
//                 row offsets per seed, all within the seed's R + 1) -- and
//                 a seed whose rows do not rise strictly, or with a hit
//                 outside its (frame, sector), is refused before the fit;
//                 during the fit each next row is resolved a step ahead.
//                 ERRS: hit h is measured with variances err[h]^2.
//  smooth_tracks  thread per seed, after the fit over rows: the state at
//                 every hit's plane from all hits.  The reference starts
//                 at the outermost plane from the fit's final state (FP64,
//                 from the fit kernel) -- one helix step, or plane by plane
//                 with the energy loss taken away -- and runs inwards by the
//                 fit's own step; along it a Kalman filter of the deviation
//                 runs inwards (Jacobians, scattering and straggling noise
//                 taken on the reference, diffuse start, the hits the fit
//                 used; rows as the fit stored them), storing per hit the
//                 filtered deviation, its covariance, the reference and the
//                 step that arrived there (Jacobian, noise, energy-loss
//                 factors; 38 doubles, 16-byte stores); then the
//                 Rauch-Tung-Striebel pass outwards reads them back (no
//                 step is taken again) and solves with P = F (C + Q) F^T
//                 by a Cholesky factorisation.
#include "tpc_fit_common.hpp"
#include "tpc_fit_ms.hpp"

namespace {

struct MsArgs {
    FitArgs F;
    double kbz;            // -c Bz in double precision
    double x0, mass2, cut;
    bool scatter;          // x0 finite
    bool eloss;            // rho > 0
    double mass, rho, zoa;         // energy loss: mass, density, Z/A,
    double inv_mass2, me_over_m, inv_exc2;   // 1/m^2, m_e/m, 1/I^2
    uint8_t *rejected;     // [cap_hits] or null
    // fits over any rows
    const int32_t *row_offsets;   // cluster layout of the frames
    const int32_t *frame;         // frame of each seed
    int32_t n_frames;
    const float2 *err;            // per-cluster (sigma_y, sigma_z), cm
    double *pfin;                 // [cap_seeds][5] final state in FP64, or null
    int16_t *rows_out;            // [cap_hits] row of every seed hit (ROWS), or null
};

// The segment of plane distance dx about to be crossed, seen from the
// state p at the plane the step leaves: path ds = |dx| sqrt(1+t^2) /
// sqrt(1-s^2), momentum P = sqrt(1+t^2)/|w|, energy E, beta^2 = P^2/E^2.
struct Segment {
    double ds, P, E, b2;
};

__device__ inline Segment segment(const MsArgs &A, const double p[5], double dx) {
    const double s = p[2], t = p[3], w = p[4];
    const double st = sqrt(1.0 + t * t);
    Segment g;
    g.ds = fabs(dx) * st / sqrt(1.0 - s * s);
    g.P = st / fabs(w);
    const double P2 = g.P * g.P;
    const double E2 = P2 + A.mass2;
    g.E = sqrt(E2);
    g.b2 = P2 / E2;
    return g;
}

// Adds the scattering of the segment to C (Highland: theta0^2 =
// (0.0136 / (beta P))^2 ds/X0 (1 + 0.038 ln(ds/X0))^2; the logarithm, which
// only scales the noise, in single precision).
__device__ inline void add_scattering(const MsArgs &A, const double p[5], const Segment &g, SymT<double> &C) {
    const double s = p[2], t = p[3], w = p[4];
    if (!A.scatter || w == 0.0) return;
    const double t2 = 1.0 + t * t;
    const double xr = g.ds / A.x0;
    const double f = 1.0 + 0.038 * (double)logf((float)xr);
    const double k = 0.0136 * 0.0136 / (g.b2 * g.P * g.P);
    const double th2 = k * xr * f * f;
    C.c22 += th2 * (1.0 - s * s) * t2;
    C.c33 += th2 * t2 * t2;
    C.c43 += th2 * t * w * t2;
    C.c44 += th2 * t * t * w * w;
}

// Energy-loss map of the segment (the particle moves outwards: dir = +1
// gives the mean loss back, a step inwards; -1 takes it away).  Mean loss
// ds rho <dE/dx> with the Bethe formula (unit charge, no density term; its
// logarithm in single precision, which changes the loss by ~1e-7 of
// itself), straggling variance of Bohr's relativistic form;
// P' = sqrt(E'^2 - m^2), w' = w P/P'.  With the loss held fixed, w' depends
// on t and w: j43 = dw'/dt, j44 = dw'/dw; vw is the straggling as variance
// of w at the start.  A segment that would change the momentum by more than
// 1 % is left alone (identity, no noise).  Returns true if the particle
// stops.
__device__ inline bool eloss_map(const MsArgs &A, const double p[5], const Segment &g, double dir, double &wo,
                                 double &j43, double &j44, double &vw) {
    const double t = p[3], w = p[4];
    wo = w;
    j43 = 0.0;
    j44 = 1.0;
    vw = 0.0;
    if (w == 0.0) return false;
    const double K = 0.307075e-3, me = 0.51099895e-3;
    const double m = A.mass, P2 = g.P * g.P;
    const double bg2 = P2 * A.inv_mass2, r = A.me_over_m;
    const double W = 2.0 * me * bg2 / (1.0 + 2.0 * (g.E / m) * r + r * r);
    const double L = (double)logf((float)(2.0 * me * bg2 * W * A.inv_exc2));
    const double dedx = K * A.zoa / g.b2 * (0.5 * L - g.b2);
    const double E1 = g.E + dir * (g.ds * A.rho * dedx);
    if (!(E1 > m)) return true;
    const double P1 = sqrt(E1 * E1 - A.mass2);
    if (fabs(P1 - g.P) > 0.01 * g.P) return false;
    const double q = g.P / P1, e = E1 / g.E;
    wo = w * q;
    j44 = q * q * q * e;
    const double t2 = 1.0 + t * t;
    j43 = wo * t / t2 * (1.0 - e * q * q);
    const double varE = K * A.zoa * A.rho * g.ds * me * (1.0 - 0.5 * g.b2) / (1.0 - g.b2);
    const double dw = w * g.E / P2;
    vw = varE * dw * dw;
    return false;
}

// C <- J C J^T for J the identity but for row 4 = (0, 0, 0, a, b).
__device__ inline void eloss_cov(SymT<double> &C, double a, double b) {
    const double c30 = C.c30, c31 = C.c31, c32 = C.c32, c33 = C.c33, c43 = C.c43, c44 = C.c44;
    C.c40 = a * c30 + b * C.c40;
    C.c41 = a * c31 + b * C.c41;
    C.c42 = a * c32 + b * C.c42;
    C.c43 = a * c33 + b * c43;
    C.c44 = a * a * c33 + 2.0 * a * b * c43 + b * b * c44;
}

// Row of cluster id at or below row r_hi of a (frame, sector) whose R + 1
// row offsets are ro: walking down from r_hi, the first row starting at or
// before id; -1 if id is not in that row (it lies above r_hi, or below the
// first row).
__device__ inline int walk_row(const int32_t *ro, int r_hi, int32_t id) {
    int r = r_hi;
    while (r >= 0 && ro[r] > id) --r;
    return (r >= 0 && id < ro[r + 1]) ? r : -1;
}

// Rows of the outermost, middle ((n-1)/2) and innermost hits of a seed, if
// every hit lies in the (frame, sector) and the rows rise strictly.
__device__ inline bool seed_rows(const int32_t *ro, int R, const SeedView &sv, int &ra, int &rb, int &rc) {
    const int n = sv.n, kb = (n - 1) / 2;
    const int32_t top = sv.hh[n - 1];
    if (top < ro[0] || top >= ro[R]) return false;
    int lo = 0, hi = R - 1;                       // ro[lo] <= top < ro[hi + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ro[mid] <= top) lo = mid;
        else hi = mid - 1;
    }
    int r = lo;
    ra = rb = r;
    for (int k = n - 2; k >= 0; --k) {
        r = walk_row(ro, r - 1, sv.hh[k]);
        if (r < 0) return false;
        if (k == kb) rb = r;
    }
    rc = r;
    return true;
}

template <bool ROWS, bool ERRS>
__device__ inline void fit_ms_one(const MsArgs &A, int i, const float *xs) {
    static_assert(ROWS || !ERRS, "per-cluster errors come with the row lookup");
    const FitArgs &F = A.F;
    SeedView sv = seed_view(F, i);
    const int32_t *ro = nullptr;
    int ra = 0, rb = 0, rc = 0;                   // rows of hits n-1, (n-1)/2, 0
    bool refused = false;
    if (ROWS) {
        // the layout gives the rows; first_row is not read
        const int32_t fi = A.frame[i];
        const bool inb = sv.n >= 3 && sv.o0 >= 0 && sv.o0 <= F.cap_hits - sv.n;
        if (inb && A.rejected)
            for (int k = 0; k < sv.n; ++k) A.rejected[sv.o0 + k] = 0;
        sv.sane = inb && sv.sec >= 0 && sv.sec < F.n_sectors && fi >= 0 && fi < A.n_frames;
        if (sv.sane) {
            ro = A.row_offsets + ((size_t)fi * F.n_sectors + sv.sec) * F.n_rows;
            sv.sane = seed_rows(ro, F.n_rows, sv, ra, rb, rc);
        }
        refused = !sv.sane;
    } else {
        if (sv.sane) {
            ra = sv.row0 + sv.n - 1;
            rb = sv.row0 + (sv.n - 1) / 2;
            rc = sv.row0;
        }
        if (sv.sane && A.rejected)
            for (int k = 0; k < sv.n; ++k) A.rejected[sv.o0 + k] = 0;
    }
    double p[5] = {0, 0, 0, 0, 0};
    SymT<double> C = {};
    double chi2 = 0.0;
    int status = TPC_FIT_OK, used = 1;
    double xcur = sv.sane ? (double)xs[ra] : 0.0;
    double vy = F.vy, vz = F.vz;
    if (ERRS && sv.sane) {
        const float2 e = A.err[sv.hh[sv.n - 1]];
        vy = (double)e.x * (double)e.x;
        vz = (double)e.y * (double)e.y;
    }
    if (!sv.sane) {
        status = TPC_FIT_INIT_FAIL;
    } else {
        const int ka = sv.n - 1, kb = (sv.n - 1) / 2;
        double ya, za, yb, zb, yc, zc;
        hit_meas(F, sv, ka, F.hyz ? 0 : sv.hh[ka], ya, za);
        hit_meas(F, sv, kb, F.hyz ? 0 : sv.hh[kb], yb, zb);
        hit_meas(F, sv, 0, F.hyz ? 0 : sv.hh[0], yc, zc);
        (void)zb;
        if (!helix_start<double, double>((double)xs[ra], ya, za, (double)xs[rb], yb, (double)xs[rc], yc, zc,
                                         A.kbz, F.max_sin, p))
            status = TPC_FIT_INIT_FAIL;
    }
    if (!refused) {
        C.c00 = vy;
        C.c11 = vz;
        C.c22 = F.var_s;
        C.c33 = F.var_t;
        C.c44 = F.var_w;
    }
    if (status == TPC_FIT_OK) {
        float2 raw = hit_raw(F, sv, sv.n - 2, F.hyz ? 0 : sv.hh[sv.n - 2]);
        int rk = ra;
        // ROWS: the row of the next hit is resolved a step ahead -- the row
        // starts one and two rows below are loaded at the top of a step and
        // compared after its helix step (a longer gap walks on); equal to
        // walk_row, as seed_rows has checked every row
        int rnext = ROWS ? walk_row(ro, ra - 1, sv.hh[sv.n - 2]) : 0;
        if (ROWS && A.rows_out) A.rows_out[sv.o0 + sv.n - 1] = (int16_t)ra;
        for (int k = sv.n - 2; k >= 0; --k) {
            double my, mz;
            hit_fix(F, sv, k, raw, my, mz);
            if (k > 0) raw = hit_raw(F, sv, k - 1, F.hyz ? 0 : sv.hh[k - 1]);
            int32_t nid = 0, v1 = INT32_MAX, v2 = INT32_MAX;
            if (ROWS) {
                rk = rnext;
                if (A.rows_out) A.rows_out[sv.o0 + k] = (int16_t)rk;
                if (k > 0) {
                    nid = sv.hh[k - 1];
                    if (rk >= 1) v1 = ro[rk - 1];
                    if (rk >= 2) v2 = ro[rk - 2];
                }
            } else {
                rk = sv.row0 + k;
            }
            if (ERRS) {
                const float2 e = A.err[sv.hh[k]];
                vy = (double)e.x * (double)e.x;
                vz = (double)e.y * (double)e.y;
            }
            const double xk = (double)xs[rk];
            const double dx = xk - xcur;
            if (A.scatter || A.eloss) {
                const Segment g = segment(A, p, dx);
                add_scattering(A, p, g, C);
                if (A.eloss) {
                    double w1, a, b, vw;
                    if (eloss_map(A, p, g, 1.0, w1, a, b, vw)) {
                        status = TPC_FIT_SIN_FAIL;
                        break;
                    }
                    C.c44 += vw;
                    eloss_cov(C, a, b);
                    p[4] = w1;
                }
            }
            StepJac J;
            if (!helix_step<double, double>(p, dx, A.kbz, F.max_sin, J)) {
                status = TPC_FIT_SIN_FAIL;
                break;
            }
            sym_transport<double, false>(C, J);
            xcur = xk;
            if (ROWS && k > 0) rnext = nid >= v1 ? rk - 1 : (nid >= v2 ? rk - 2 : walk_row(ro, rk - 3, nid));
            // predicted-residual chi2 of the hit
            const double r0 = my - p[0], r1 = mz - p[1];
            const double S00 = C.c00 + vy, S01 = C.c10, S11 = C.c11 + vz;
            const double det = S00 * S11 - S01 * S01;
            const double chi = (r0 * (S11 * r0 - S01 * r1) + r1 * (S00 * r1 - S01 * r0)) / det;
            // (a singular S is not a rejection: the update reports it)
            if (det > 0.0 && chi > A.cut) {
                if (A.rejected) A.rejected[sv.o0 + k] = 1;
                continue;
            }
            const double dchi = kalman_update<double>(p, C, my, mz, vy, vz);
            chi2 += dchi;
            const double chk = chi2 + p[0] + p[1] + p[2] + p[3] + p[4];
            if (!(dchi >= 0.0) || !(chk - chk == 0.0)) {
                status = TPC_FIT_NUM_FAIL;
                break;
            }
            ++used;
        }
    }
    if (A.pfin)
        for (int q = 0; q < 5; ++q) A.pfin[(size_t)i * 5 + q] = p[q];
    F.out.x[i] = (float)xcur;
    float *po = F.out.par + (size_t)i * 5;
    for (int q = 0; q < 5; ++q) po[q] = (float)p[q];
    float *co = F.out.cov + (size_t)i * 15;
    const double cc[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                           C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    for (int q = 0; q < 15; ++q) co[q] = (float)cc[q];
    F.out.chi2[i] = (float)chi2;
    F.out.ndf[i] = 2 * used - 5;
    F.out.status[i] = status;
}

template <bool ROWS, bool ERRS>
__global__ void __launch_bounds__(TPC_BLOCK) fit_ms_tracks(MsArgs A) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < A.F.n_rows; r += TPC_BLOCK) xs[r] = A.F.row_x[r];
    __syncthreads();
    int T = *A.F.n_seeds;
    if (T > A.F.cap_seeds) T = A.F.cap_seeds;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        fit_ms_one<ROWS, ERRS>(A, i, xs);
}

// Per seed hit the smoother keeps the filtered deviation (5), its
// covariance (15, packed), the reference state (5) and the step that
// arrived at the hit's plane from the next one out (helix Jacobian (6),
// scattering and straggling noise (4), energy-loss factors (2)), padded to
// 38 doubles.
constexpr int SM_REC = 38;

__device__ inline void load_record(const double *rec, double w[SM_REC]) {
    const double2 *v = reinterpret_cast<const double2 *>(rec);
    for (int q = 0; q < SM_REC / 2; ++q) {
        const double2 x = v[q];
        w[2 * q] = x.x;
        w[2 * q + 1] = x.y;
    }
}

struct SmArgs {
    MsArgs M;
    SmWs w;
    const uint8_t *rej;
    float *hit_par, *hit_cov;
};

__device__ inline void sym_add(SymT<double> &C, const SymT<double> &Q) {
    C.c00 += Q.c00; C.c10 += Q.c10; C.c11 += Q.c11; C.c20 += Q.c20; C.c21 += Q.c21;
    C.c22 += Q.c22; C.c30 += Q.c30; C.c31 += Q.c31; C.c32 += Q.c32; C.c33 += Q.c33;
    C.c40 += Q.c40; C.c41 += Q.c41; C.c42 += Q.c42; C.c43 += Q.c43; C.c44 += Q.c44;
}

__device__ inline void sym_dense(const SymT<double> &C, double M[5][5]) {
    const double v[15] = {C.c00, C.c10, C.c11, C.c20, C.c21, C.c22, C.c30, C.c31,
                          C.c32, C.c33, C.c40, C.c41, C.c42, C.c43, C.c44};
    int q = 0;
    for (int r = 0; r < 5; ++r)
        for (int c = 0; c <= r; ++c, ++q) M[r][c] = M[c][r] = v[q];
}

__device__ inline SymT<double> sym_packed(const double M[5][5]) {
    SymT<double> C;
    C.c00 = M[0][0]; C.c10 = M[1][0]; C.c11 = M[1][1]; C.c20 = M[2][0]; C.c21 = M[2][1];
    C.c22 = M[2][2]; C.c30 = M[3][0]; C.c31 = M[3][1]; C.c32 = M[3][2]; C.c33 = M[3][3];
    C.c40 = M[4][0]; C.c41 = M[4][1]; C.c42 = M[4][2]; C.c43 = M[4][3]; C.c44 = M[4][4];
    return C;
}

// d <- F d for the step Jacobian (identity plus the six off-diagonal terms).
__device__ inline void jac_apply(const StepJac &J, const double d[5], double o[5]) {
    o[0] = d[0] + J.f02 * d[2] + J.f04 * d[4];
    o[1] = d[1] + J.f12 * d[2] + J.f13 * d[3] + J.f14 * d[4];
    o[2] = d[2] + J.f24 * d[4];
    o[3] = d[3];
    o[4] = d[4];
}

// A = F C (dense) for the step Jacobian.
__device__ inline void jac_times(const StepJac &J, const double C[5][5], double A[5][5]) {
    for (int c = 0; c < 5; ++c) {
        A[0][c] = C[0][c] + J.f02 * C[2][c] + J.f04 * C[4][c];
        A[1][c] = C[1][c] + J.f12 * C[2][c] + J.f13 * C[3][c] + J.f14 * C[4][c];
        A[2][c] = C[2][c] + J.f24 * C[4][c];
        A[3][c] = C[3][c];
        A[4][c] = C[4][c];
    }
}

// Solves P X = A (P symmetric positive definite, 5x5) in place of A by a
// Cholesky factorisation; false if a pivot is not positive.
__device__ inline bool chol_solve(double P[5][5], double A[5][5]) {
    for (int j = 0; j < 5; ++j) {
        double s = P[j][j];
        for (int k = 0; k < j; ++k) s -= P[j][k] * P[j][k];
        if (!(s > 0.0)) return false;
        const double l = sqrt(s);
        P[j][j] = l;
        for (int r = j + 1; r < 5; ++r) {
            double t = P[r][j];
            for (int k = 0; k < j; ++k) t -= P[r][k] * P[j][k];
            P[r][j] = t / l;
        }
    }
    for (int c = 0; c < 5; ++c) {
        for (int r = 0; r < 5; ++r) {           // L y = a
            double t = A[r][c];
            for (int k = 0; k < r; ++k) t -= P[r][k] * A[k][c];
            A[r][c] = t / P[r][r];
        }
        for (int r = 4; r >= 0; --r) {          // L^T x = y
            double t = A[r][c];
            for (int k = r + 1; k < 5; ++k) t -= P[k][r] * A[k][c];
            A[r][c] = t / P[r][r];
        }
    }
    return true;
}

template <bool ERRS>
__device__ inline void smooth_one(const SmArgs &S, int i, const float *xs) {
    const MsArgs &A = S.M;
    const FitArgs &F = A.F;
    const SeedView sv = seed_view(F, i);
    const int n = sv.n;
    if (!(n >= 3 && sv.o0 >= 0 && sv.o0 <= F.cap_hits - n)) return;
    float *hp = S.hit_par + (size_t)sv.o0 * 5;
    float *hc = S.hit_cov + (size_t)sv.o0 * 15;
    int status = F.out.status[i];
    if (status == TPC_FIT_OK) {
        // the fit accepted the seed and stored the row of every hit
        const double *pf = S.w.pfin + (size_t)i * 5;
        double *wd = S.w.wd + (size_t)sv.o0 * SM_REC;
        const int16_t *wr = S.w.wrow + sv.o0;
        const int ra = wr[n - 1], rc = wr[0];
        const uint8_t *rej = S.rej + sv.o0;
        // the reference at the outermost plane: one helix step from the fit's
        // final state, or, with energy loss, plane by plane taking the loss away
        double R[5];
        for (int q = 0; q < 5; ++q) R[q] = pf[q];
        StepJac J;
        if (A.eloss) {
            for (int k = 1; k < n && status == TPC_FIT_OK; ++k) {
                const double dx = (double)xs[wr[k]] - (double)xs[wr[k - 1]];
                double w1 = R[4], a, b, vw;
                if (!helix_step<double, double>(R, dx, A.kbz, F.max_sin, J) ||
                    eloss_map(A, R, segment(A, R, dx), -1.0, w1, a, b, vw))
                    status = TPC_FIT_SIN_FAIL;
                R[4] = w1;
            }
        } else if (!helix_step<double, double>(R, (double)xs[ra] - (double)xs[rc], A.kbz, F.max_sin, J)) {
            status = TPC_FIT_SIN_FAIL;
        }
        double vy = F.vy, vz = F.vz;
        if (ERRS) {
            const float2 e = A.err[sv.hh[n - 1]];
            vy = (double)e.x * (double)e.x;
            vz = (double)e.y * (double)e.y;
        }
        // inwards along the reference: Kalman filter of the deviation d
        double d[5] = {0, 0, 0, 0, 0};
        SymT<double> C = {};
        C.c00 = 1e4 * vy;
        C.c11 = 1e4 * vz;
        C.c22 = F.var_s;
        C.c33 = F.var_t;
        C.c44 = F.var_w;
        int rk = ra;
        int rn = wr[n - 2];                 // loaded a step ahead
        for (int k = n - 1; k >= 0 && status == TPC_FIT_OK; --k) {
            // the step that arrives at plane k: its noise and energy-loss
            // factors, kept for the outward pass with its Jacobian J
            SymT<double> Q = {};
            double ea = 0.0, eb = 1.0;
            if (k < n - 1) {
                const int rcur = rn;
                if (k > 0) rn = wr[k - 1];
                const double dx = (double)xs[rcur] - (double)xs[rk];
                const Segment g = (A.scatter || A.eloss) ? segment(A, R, dx) : Segment{};
                add_scattering(A, R, g, Q);
                if (A.eloss) {
                    double w1, vw;
                    if (eloss_map(A, R, g, 1.0, w1, ea, eb, vw)) {
                        status = TPC_FIT_SIN_FAIL;
                        break;
                    }
                    Q.c44 += vw;
                    sym_add(C, Q);
                    eloss_cov(C, ea, eb);
                    d[4] = ea * d[3] + eb * d[4];
                    R[4] = w1;
                } else {
                    sym_add(C, Q);
                }
                if (!helix_step<double, double>(R, dx, A.kbz, F.max_sin, J)) {
                    status = TPC_FIT_SIN_FAIL;
                    break;
                }
                double nd[5];
                jac_apply(J, d, nd);
                for (int q = 0; q < 5; ++q) d[q] = nd[q];
                sym_transport<double, false>(C, J);
                rk = rcur;
                if (ERRS) {
                    const float2 e = A.err[sv.hh[k]];
                    vy = (double)e.x * (double)e.x;
                    vz = (double)e.y * (double)e.y;
                }
            }
            if (!rej[k]) {
                double my, mz;
                hit_meas(F, sv, k, F.hyz ? 0 : sv.hh[k], my, mz);
                const double dchi = kalman_update<double>(d, C, my - R[0], mz - R[1], vy, vz);
                const double chk = dchi + d[0] + d[1] + d[2] + d[3] + d[4];
                if (!(chk - chk == 0.0)) {
                    status = TPC_FIT_NUM_FAIL;
                    break;
                }
            }
            // d, C, the reference and the arriving step (Jacobian, the four
            // noise terms, energy-loss factors): 38 doubles as 19 16-byte
            // stores (the record is 16-byte aligned)
            double2 *w = reinterpret_cast<double2 *>(wd + (size_t)k * SM_REC);
            w[0] = make_double2(d[0], d[1]);
            w[1] = make_double2(d[2], d[3]);
            w[2] = make_double2(d[4], C.c00);
            w[3] = make_double2(C.c10, C.c11);
            w[4] = make_double2(C.c20, C.c21);
            w[5] = make_double2(C.c22, C.c30);
            w[6] = make_double2(C.c31, C.c32);
            w[7] = make_double2(C.c33, C.c40);
            w[8] = make_double2(C.c41, C.c42);
            w[9] = make_double2(C.c43, C.c44);
            w[10] = make_double2(R[0], R[1]);
            w[11] = make_double2(R[2], R[3]);
            w[12] = make_double2(R[4], J.f02);
            w[13] = make_double2(J.f04, J.f12);
            w[14] = make_double2(J.f13, J.f14);
            w[15] = make_double2(J.f24, Q.c22);
            w[16] = make_double2(Q.c33, Q.c43);
            w[17] = make_double2(Q.c44, ea);
            w[18] = make_double2(eb, 0.0);
        }
        // outwards: Rauch-Tung-Striebel
        if (status == TPC_FIT_OK) {
            double ds[5], Cs[5][5];
            // the step from plane 1 to plane 0 is stored with plane 0
            StepJac Jk;
            double q22, q33, q43, q44, ea, eb;
            {
                double w[SM_REC];
                load_record(wd, w);
                Jk = StepJac{w[25], w[26], w[27], w[28], w[29], w[30]};
                q22 = w[31]; q33 = w[32]; q43 = w[33]; q44 = w[34]; ea = w[35]; eb = w[36];
                for (int q = 0; q < 5; ++q) ds[q] = w[q];
                SymT<double> C0;
                C0.c00 = w[5]; C0.c10 = w[6]; C0.c11 = w[7]; C0.c20 = w[8]; C0.c21 = w[9];
                C0.c22 = w[10]; C0.c30 = w[11]; C0.c31 = w[12]; C0.c32 = w[13]; C0.c33 = w[14];
                C0.c40 = w[15]; C0.c41 = w[16]; C0.c42 = w[17]; C0.c43 = w[18]; C0.c44 = w[19];
                sym_dense(C0, Cs);
                for (int q = 0; q < 5; ++q) hp[q] = (float)(w[20 + q] + ds[q]);
            }
            {
                const SymT<double> P0 = sym_packed(Cs);
                const double cc[15] = {P0.c00, P0.c10, P0.c11, P0.c20, P0.c21, P0.c22, P0.c30, P0.c31,
                                       P0.c32, P0.c33, P0.c40, P0.c41, P0.c42, P0.c43, P0.c44};
                for (int q = 0; q < 15; ++q) hc[q] = (float)cc[q];
            }
            for (int k = 1; k < n; ++k) {
                double w[SM_REC];
                load_record(wd + (size_t)k * SM_REC, w);
                const double dk[5] = {w[0], w[1], w[2], w[3], w[4]};
                SymT<double> Ck;
                Ck.c00 = w[5]; Ck.c10 = w[6]; Ck.c11 = w[7]; Ck.c20 = w[8]; Ck.c21 = w[9];
                Ck.c22 = w[10]; Ck.c30 = w[11]; Ck.c31 = w[12]; Ck.c32 = w[13]; Ck.c33 = w[14];
                Ck.c40 = w[15]; Ck.c41 = w[16]; Ck.c42 = w[17]; Ck.c43 = w[18]; Ck.c44 = w[19];
                const double Rk[5] = {w[20], w[21], w[22], w[23], w[24]};
                // the step inwards from plane k: F = Jh Je, noise Q (stored
                // with plane k - 1 by the filter)
                SymT<double> Pq = Ck;
                Pq.c22 += q22;
                Pq.c33 += q33;
                Pq.c43 += q43;
                Pq.c44 += q44;
                double Cd[5][5], X[5][5], ed[5] = {dk[0], dk[1], dk[2], dk[3], dk[4]};
                sym_dense(Ck, Cd);
                if (A.eloss) {
                    eloss_cov(Pq, ea, eb);
                    ed[4] = ea * dk[3] + eb * dk[4];
                    double EC[5][5];
                    for (int a = 0; a < 5; ++a)
                        for (int b = 0; b < 5; ++b)
                            EC[a][b] = a < 4 ? Cd[a][b] : ea * Cd[3][b] + eb * Cd[4][b];
                    jac_times(Jk, EC, X);                    // F C_k
                } else {
                    jac_times(Jk, Cd, X);                    // F C_k
                }
                sym_transport<double, false>(Pq, Jk);       // P = F (C_k + Q) F^T
                double P[5][5], Pd[5][5];
                sym_dense(Pq, P);
                sym_dense(Pq, Pd);
                if (!chol_solve(P, X)) {                     // X = P^-1 F C_k = G^T
                    status = TPC_FIT_NUM_FAIL;
                    break;
                }
                double pd[5], e[5], nds[5];
                jac_apply(Jk, ed, pd);
                for (int q = 0; q < 5; ++q) e[q] = ds[q] - pd[q];
                for (int a = 0; a < 5; ++a) {
                    double acc = dk[a];
                    for (int b = 0; b < 5; ++b) acc += X[b][a] * e[b];
                    nds[a] = acc;
                }
                // Cs <- C_k + G (Cs - P) G^T
                double D[5][5], T[5][5];
                for (int a = 0; a < 5; ++a)
                    for (int b = 0; b < 5; ++b) D[a][b] = Cs[a][b] - Pd[a][b];
                for (int a = 0; a < 5; ++a)
                    for (int b = 0; b < 5; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < 5; ++c) acc += X[c][a] * D[c][b];
                        T[a][b] = acc;
                    }
                for (int a = 0; a < 5; ++a)
                    for (int b = 0; b <= a; ++b) {
                        double acc = 0.0;
                        for (int c = 0; c < 5; ++c) acc += T[a][c] * X[c][b];
                        Cs[a][b] = Cs[b][a] = Cd[a][b] + acc;
                    }
                for (int q = 0; q < 5; ++q) ds[q] = nds[q];
                float *o = hp + (size_t)k * 5;
                for (int q = 0; q < 5; ++q) o[q] = (float)(Rk[q] + ds[q]);
                float *oc = hc + (size_t)k * 15;
                int q = 0;
                for (int a = 0; a < 5; ++a)
                    for (int b = 0; b <= a; ++b, ++q) oc[q] = (float)Cs[a][b];
                // the step from plane k + 1, stored with plane k
                Jk = StepJac{w[25], w[26], w[27], w[28], w[29], w[30]};
                q22 = w[31]; q33 = w[32]; q43 = w[33]; q44 = w[34]; ea = w[35]; eb = w[36];
            }
        }
        if (status != TPC_FIT_OK) F.out.status[i] = status;
    }
    if (status != TPC_FIT_OK) {
        for (int k = 0; k < n; ++k) {
            for (int q = 0; q < 5; ++q) hp[(size_t)k * 5 + q] = 0.f;
            for (int q = 0; q < 15; ++q) hc[(size_t)k * 15 + q] = 0.f;
        }
    }
}

template <bool ERRS>
__global__ void __launch_bounds__(TPC_BLOCK) smooth_tracks(SmArgs S) {
    __shared__ float xs[TPC_MAX_ROWS];
    for (int r = threadIdx.x; r < S.M.F.n_rows; r += TPC_BLOCK) xs[r] = S.M.F.row_x[r];
    __syncthreads();
    int T = *S.M.F.n_seeds;
    if (T > S.M.F.cap_seeds) T = S.M.F.cap_seeds;
    for (int i = blockIdx.x * TPC_BLOCK + threadIdx.x; i < T; i += gridDim.x * TPC_BLOCK)
        smooth_one<ERRS>(S, i, xs);
}

MsArgs make_ms_args(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const tpc_material *mat,
                    const tpc_tracks *tr, uint8_t *rejected, void *ws, hipStream_t st) {
    MsArgs A;
    A.F = make_fit_args(ctx, fr, sd, nullptr);
    A.F.out = *tr;
    if (sd->hit_yz) {
        A.F.hyz = reinterpret_cast<const float2 *>(sd->hit_yz);
    } else {
        float2 *hyz;
        fit_ws_layout(ws, sd->cap_seeds, sd->cap_hits, nullptr, &hyz);
        A.F.hyz = hyz;
        (void)launch_gather(fr, sd, hyz, st);    // a launch error surfaces at the fit's launch
    }
    A.kbz = -0.00299792458 * (double)ctx->cfg.bz;
    A.x0 = mat ? (double)mat->x0 : (double)INFINITY;
    A.scatter = mat && mat->x0 < INFINITY;
    A.mass2 = mat ? (double)mat->mass * (double)mat->mass : 0.0;
    A.cut = mat ? (double)mat->chi2_cut : (double)INFINITY;
    A.eloss = mat && mat->rho > 0.f;
    A.mass = mat ? (double)mat->mass : 0.0;
    A.rho = mat ? (double)mat->rho : 0.0;
    A.zoa = mat ? (double)mat->z_over_a : 0.0;
    A.inv_mass2 = A.eloss ? 1.0 / A.mass2 : 0.0;
    A.me_over_m = A.eloss ? 0.51099895e-3 / A.mass : 0.0;
    A.inv_exc2 = A.eloss ? 1.0 / ((double)mat->mean_exc * (double)mat->mean_exc) : 0.0;
    A.rejected = rejected;
    A.row_offsets = fr->row_offsets;
    A.frame = sd->frame;
    A.n_frames = fr->n_frames;
    A.err = nullptr;
    A.pfin = nullptr;
    A.rows_out = nullptr;
    return A;
}

int fit_blocks(const tpc_seeds *sd) {
    int blocks = (sd->cap_seeds + TPC_BLOCK - 1) / TPC_BLOCK;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace

hipError_t launch_fit_material(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd,
                               const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected,
                               void *ws, hipStream_t st) {
    const MsArgs A = make_ms_args(ctx, fr, sd, mat, tr, rejected, ws, st);
    hipLaunchKernelGGL((fit_ms_tracks<false, false>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_fit_rows(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const float *err,
                           const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected, void *ws,
                           hipStream_t st) {
    MsArgs A = make_ms_args(ctx, fr, sd, mat, tr, rejected, ws, st);
    A.err = reinterpret_cast<const float2 *>(err);
    if (err)
        hipLaunchKernelGGL((fit_ms_tracks<true, true>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    else
        hipLaunchKernelGGL((fit_ms_tracks<true, false>), dim3(fit_blocks(sd)), dim3(TPC_BLOCK), 0, st, A);
    return hipGetLastError();
}

size_t smooth_ws_layout(void *ws, int64_t cap_seeds, int64_t cap_hits, SmWs *out) {
    const size_t fb = fit_ws_layout(nullptr, cap_seeds, cap_hits, nullptr, nullptr);
    WsCarver w(ws ? (void *)((char *)ws + fb) : nullptr);
    double *pfin = w.take<double>((size_t)(cap_seeds > 0 ? cap_seeds : 1) * 5);
    double *wd = w.take<double>((size_t)(cap_hits > 0 ? cap_hits : 1) * SM_REC);
    int16_t *wrow = w.take<int16_t>((size_t)(cap_hits > 0 ? cap_hits : 1));
    if (out) *out = SmWs{pfin, wd, wrow};
    return fb + ((w.off + 255) & ~size_t(255));
}

hipError_t launch_smooth(const tpc_context *ctx, const tpc_frames *fr, const tpc_seeds *sd, const float *err,
                         const tpc_material *mat, const tpc_tracks *tr, uint8_t *rejected, float *hit_par,
                         float *hit_cov, void *ws, hipStream_t st) {
    SmArgs S;
    S.M = make_ms_args(ctx, fr, sd, mat, tr, rejected, ws, st);
    S.M.err = reinterpret_cast<const float2 *>(err);
    smooth_ws_layout(ws, sd->cap_seeds, sd->cap_hits, &S.w);
    S.M.pfin = S.w.pfin;
    S.M.rows_out = S.w.wrow;
    S.rej = rejected;
    S.hit_par = hit_par;
    S.hit_cov = hit_cov;
    const int blocks = fit_blocks(sd);
    if (err) {
        hipLaunchKernelGGL((fit_ms_tracks<true, true>), dim3(blocks), dim3(TPC_BLOCK), 0, st, S.M);
        hipLaunchKernelGGL((smooth_tracks<true>), dim3(blocks), dim3(TPC_BLOCK), 0, st, S);
    } else {
        hipLaunchKernelGGL((fit_ms_tracks<true, false>), dim3(blocks), dim3(TPC_BLOCK), 0, st, S.M);
        hipLaunchKernelGGL((smooth_tracks<false>), dim3(blocks), dim3(TPC_BLOCK), 0, st, S);
    }
    return hipGetLastError();
}
