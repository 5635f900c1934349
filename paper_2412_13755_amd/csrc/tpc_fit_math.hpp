// Helix-fit arithmetic shared by the forward fit and its adjoint.
//
// State p = (y, z, s = sin phi, t = tan lambda, w = q/pT) on a pad-row plane
// x, track oriented towards +x, curvature kappa = -c Bz w (counter-clockwise
// positive); covariance as the 15 entries of its lower triangle.
//
// Precision.  The forward filter (state, helix transport, Jacobian,
// covariance transport F C F^T and Kalman update) runs in the type R, double
// in the library: a short track's curvature is fixed by sub-micron
// sagittas, so single-precision transport of y alone moves q/pT by ~1e-4
// relative, and a single-precision covariance update loses up to all
// significant digits when the diffuse start covariance collapses onto the
// first hits (C - K H C cancels).  On gfx950 the FP64 vector FMA issues at the
// rate of the non-packed FP32 one, so double costs no more than float here.
// Reciprocals and square roots in the inner loop use the hardware estimates
// refined by Newton steps rather than the correctly rounded sequences.  The
// second-order term of the adjoint (derivative of the Jacobian) is evaluated
// in single precision.
// No MFMA: a 5x5 symmetric update is not a dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#define TPC_C_LIGHT 0.00299792458f

template <class R>
struct SymT {
    // lower triangle, row by row: 00 10 11 20 21 22 30 31 32 33 40 41 42 43 44
    R c00, c10, c11, c20, c21, c22, c30, c31, c32, c33, c40, c41, c42, c43, c44;
};

__host__ __device__ inline float asin_over(float u) {
    // asin(u)/u, Taylor series to u^8 near 0
    if (fabsf(u) < 0.05f) {
        float u2 = u * u;
        return 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f + u2 * (35.0f / 1152.0f))));
    }
    return asinf(u) / u;
}

// first derivative of asin(u)/u
__host__ __device__ inline float asin_over_d(float u) {
    if (fabsf(u) < 0.05f) {
        float u2 = u * u;
        return u * (1.0f / 3.0f + u2 * (3.0f / 10.0f + u2 * (15.0f / 56.0f + u2 * (35.0f / 144.0f))));
    }
    return (u / sqrtf((1.0f - u) * (1.0f + u)) - asinf(u)) / (u * u);
}

// second derivative of asin(u)/u: (1-u^2)^(-3/2) - 2 g'(u)/u
__host__ __device__ inline float asin_over_dd(float u) {
    if (fabsf(u) < 0.05f) {
        float u2 = u * u;
        return 1.0f / 3.0f + u2 * (9.0f / 10.0f + u2 * (75.0f / 56.0f + u2 * (245.0f / 144.0f)));
    }
    const float w = 1.0f / sqrtf((1.0f - u) * (1.0f + u));
    return w * w * w - 2.0f * asin_over_d(u) / u;
}

// Jacobian entries that differ from the identity.
struct StepJac {
    double f02, f04, f12, f13, f14, f24;
};

// Reciprocal and square root of positive, finite, normal doubles for the
// filter's inner loop.  On the device: the hardware estimates refined by
// Newton-Raphson (reciprocal, two steps) and by one coupled Goldschmidt step
// plus one Newton correction (square root); relative error far below the
// 1e-12 the filter needs, but not correctly rounded.  On the host: the
// library operations.
__host__ __device__ inline double recip_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// sqrt(x), and 1/sqrt(x) in *inv (the latter to about 1e-13 relative).
__host__ __device__ inline double sqrt_pos(double x, double *inv) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    if (inv) *inv = h + h;
    return g;
#else
    const double g = sqrt(x);
    if (inv) *inv = 1.0 / g;
    return g;
#endif
}

// asin(u)/u and its derivative away from 0 (|u| >= 0.05: a step that turns
// the track by more than ~6 degrees).  Out of line: rarely taken, and the
// library asin would otherwise occupy registers in the filter loop.
__host__ __device__ __attribute__((noinline)) inline double asin_over_far(double u) {
    return asin(u) / u;
}
__host__ __device__ __attribute__((noinline)) inline double asin_over_d_far(double u) {
    return (u / sqrt((1.0 - u) * (1.0 + u)) - asin(u)) / (u * u);
}

// asin(u)/u in the state precision (Taylor series to u^8 near 0)
template <class R>
__host__ __device__ inline R asin_over_r(R u) {
    if (fabs(u) < (R)0.05) {
        const R u2 = u * u;
        return (R)1 + u2 * ((R)1 / 6 + u2 * ((R)3 / 40 + u2 * ((R)5 / 112 + u2 * ((R)35 / 1152))));
    }
    return (R)asin_over_far((double)u);
}

// first derivative of asin(u)/u in the state precision
template <class R>
__host__ __device__ inline R asin_over_d_r(R u) {
    if (fabs(u) < (R)0.05) {
        const R u2 = u * u;
        return u * ((R)1 / 3 + u2 * ((R)3 / 10 + u2 * ((R)15 / 56 + u2 * ((R)35 / 144))));
    }
    return (R)asin_over_d_far((double)u);
}

// Exact helix step from x to x + dx, state and Jacobian in precision R
// (double in the library: on gfx950 the FP64 vector FMA issues at the rate
// of the non-packed FP32 one, so a single-precision Jacobian would only add
// conversions).  Returns false when |sin phi| reaches max_sin before or
// after the step; the step is evaluated regardless (no early exit keeps the
// filter loop free of branches), so p and J are then meaningless.
// The plane distance dx and kbz = -c Bz come in precision K: single in the
// fit (adjacent planes), double where steps cross several planes.
template <class R, class K = float>
__host__ __device__ inline bool helix_step(R p[5], K dx, K kbz, float max_sin, StepJac &J) {
    // kbz = -c Bz, so kappa = kbz * w
    const R s = p[2], t = p[3], w = p[4];
    const R kap = (R)kbz * w;
    const R s2 = s + kap * (R)dx;
    const bool ok = fabs(s) < (R)max_sin && fabs(s2) < (R)max_sin;
    R ic1, ic2, isq;
    const R c1 = sqrt_pos(((R)1 - s) * ((R)1 + s), &ic1);
    const R c2 = sqrt_pos(((R)1 - s2) * ((R)1 + s2), &ic2);
    const R den = c1 + c2;
    const R iden = recip_pos(den);
    const R A1 = s + s2;
    const R T = A1 * iden;                        // tan of the chord direction
    const R adx = fabs((R)dx);
    const R sq = sqrt_pos((R)1 + T * T, &isq);
    const R chord = adx * sq;
    const R u = (R)0.5 * kap * chord;
    const R sgn = dx >= (K)0 ? (R)1 : (R)-1;
    const R arc = sgn * chord * asin_over_r(u);  // signed transverse path length
    // Jacobian
    const R iden2 = iden * iden;
    const R dTs_p = (den + A1 * s * ic1) * iden2;
    const R dTs2_p = (den + A1 * s2 * ic2) * iden2;
    const R dT_ds = dTs_p + dTs2_p;
    const R dT_dw = dTs2_p * (R)dx * (R)kbz;
    R darc_dchord;                                // d(chord g(u))/dchord = 1/sqrt(1 - u^2)
    sqrt_pos(((R)1 - u) * ((R)1 + u), &darc_dchord);
    darc_dchord *= sgn;
    const R darc_dkap = sgn * (R)0.5 * chord * chord * asin_over_d_r(u);
    const R dchord_dT = adx * T * isq;
    const R q = darc_dchord * dchord_dT;
    J.f02 = (R)dx * dT_ds;
    J.f04 = (R)dx * dT_dw;
    J.f12 = t * q * dT_ds;
    J.f13 = arc;
    J.f14 = t * (q * dT_dw + darc_dkap * (R)kbz);
    J.f24 = (R)dx * (R)kbz;
    p[0] += (R)dx * T;
    p[1] += t * arc;
    p[2] = s2;
    return ok;
}

// Symmetric transport with the sparse step Jacobian F = I + N:
//   transposed == false:  C <- F C F^T
//   transposed == true:   C <- F^T C F
template <class R, bool transposed>
__host__ __device__ inline void sym_transport(SymT<R> &C, const StepJac &J) {
    const R f02 = J.f02, f04 = J.f04, f12 = J.f12, f13 = J.f13, f14 = J.f14, f24 = J.f24;
    const R C00 = C.c00, C01 = C.c10, C02 = C.c20, C03 = C.c30, C04 = C.c40;
    const R C11 = C.c11, C12 = C.c21, C13 = C.c31, C14 = C.c41;
    const R C22 = C.c22, C23 = C.c32, C24 = C.c42;
    const R C33 = C.c33, C34 = C.c43, C44 = C.c44;
    if (!transposed) {
        // A = F C: rows 0..2 change, rows 3, 4 are those of C
        const R A00 = C00 + f02 * C02 + f04 * C04;
        const R A02 = C02 + f02 * C22 + f04 * C24;
        const R A04 = C04 + f02 * C24 + f04 * C44;
        const R A10 = C01 + f12 * C02 + f13 * C03 + f14 * C04;
        const R A11 = C11 + f12 * C12 + f13 * C13 + f14 * C14;
        const R A12 = C12 + f12 * C22 + f13 * C23 + f14 * C24;
        const R A13 = C13 + f12 * C23 + f13 * C33 + f14 * C34;
        const R A14 = C14 + f12 * C24 + f13 * C34 + f14 * C44;
        const R A20 = C02 + f24 * C04;
        const R A22 = C22 + f24 * C24;
        const R A24 = C24 + f24 * C44;
        // C' = A F^T
        C.c00 = A00 + f02 * A02 + f04 * A04;
        C.c10 = A10 + f02 * A12 + f04 * A14;
        C.c11 = A11 + f12 * A12 + f13 * A13 + f14 * A14;
        C.c20 = A20 + f02 * A22 + f04 * A24;
        C.c21 = (C12 + f24 * C14) + f12 * A22 + f13 * (C23 + f24 * C34) + f14 * A24;
        C.c22 = A22 + f24 * A24;
        C.c30 = C03 + f02 * C23 + f04 * C34;
        C.c31 = C13 + f12 * C23 + f13 * C33 + f14 * C34;
        C.c32 = C23 + f24 * C34;
        C.c40 = C04 + f02 * C24 + f04 * C44;
        C.c41 = C14 + f12 * C24 + f13 * C34 + f14 * C44;
        C.c42 = C24 + f24 * C44;
        // c33, c43, c44 unchanged
    } else {
        // Q = C F: columns 2..4 change (col2 += f02 col0 + f12 col1,
        // col3 += f13 col1, col4 += f04 col0 + f14 col1 + f24 col2)
        // then C' = F^T Q: rows change the same way.
        const R Q02 = C02 + f02 * C00 + f12 * C01;
        const R Q12 = C12 + f02 * C01 + f12 * C11;
        const R Q22 = C22 + f02 * C02 + f12 * C12;
        const R Q32 = C23 + f02 * C03 + f12 * C13;
        const R Q42 = C24 + f02 * C04 + f12 * C14;
        const R Q03 = C03 + f13 * C01;
        const R Q13 = C13 + f13 * C11;
        const R Q23 = C23 + f13 * C12;
        const R Q33 = C33 + f13 * C13;
        const R Q43 = C34 + f13 * C14;
        const R Q04 = C04 + f04 * C00 + f14 * C01 + f24 * C02;
        const R Q14 = C14 + f04 * C01 + f14 * C11 + f24 * C12;
        const R Q24 = C24 + f04 * C02 + f14 * C12 + f24 * C22;
        const R Q34 = C34 + f04 * C03 + f14 * C13 + f24 * C23;
        const R Q44 = C44 + f04 * C04 + f14 * C14 + f24 * C24;
        // rows 0, 1 of F^T Q are rows 0, 1 of Q
        C.c20 = Q02;
        C.c21 = Q12;
        C.c22 = Q22 + f02 * Q02 + f12 * Q12;
        C.c30 = Q03;
        C.c31 = Q13;
        C.c32 = Q23 + f02 * Q03 + f12 * Q13;
        C.c33 = Q33 + f13 * Q13;
        C.c40 = Q04;
        C.c41 = Q14;
        C.c42 = Q24 + f02 * Q04 + f12 * Q14;
        C.c43 = Q34 + f13 * Q14;
        C.c44 = Q44 + f04 * Q04 + f14 * Q14 + f24 * Q24;
        (void)Q32; (void)Q42; (void)Q43;
        // c00, c10, c11 unchanged
    }
}

// Kalman update with measurement (my, mz), in two halves: kalman_gain forms
// the gain K = C H^T S^-1 from the predicted covariance, updates the state
// and returns the chi2 increment (negative if the residual covariance is not
// positive definite; everything is evaluated regardless, and p, C are then
// meaningless); kalman_cov applies C -= K H C.  The filter loop runs the
// covariance half of one step next to the helix step of the next, which
// does not need it.  K and the rows H C are kept in a Gain.
template <class R>
struct Gain {
    R k00, k01, k10, k11, k20, k21, k30, k31, k40, k41;   // K
    R r00, r01, r02, r03, r04, r11, r12, r13, r14;         // rows 0 and 1 of C
};

template <class R>
__host__ __device__ inline R kalman_gain(R p[5], const SymT<R> &C, R my, R mz, R vy, R vz, Gain<R> &G) {
    const R r0 = my - p[0], r1 = mz - p[1];
    const R S00 = C.c00 + vy, S01 = C.c10, S11 = C.c11 + vz;
    const R det = S00 * S11 - S01 * S01;
    const bool pd = det > (R)0;
    const R idet = recip_pos(det);
    const R i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
    // K = C[:, 0:2] S^-1
    G.k00 = C.c00 * i00 + C.c10 * i01; G.k01 = C.c00 * i01 + C.c10 * i11;
    G.k10 = C.c10 * i00 + C.c11 * i01; G.k11 = C.c10 * i01 + C.c11 * i11;
    G.k20 = C.c20 * i00 + C.c21 * i01; G.k21 = C.c20 * i01 + C.c21 * i11;
    G.k30 = C.c30 * i00 + C.c31 * i01; G.k31 = C.c30 * i01 + C.c31 * i11;
    G.k40 = C.c40 * i00 + C.c41 * i01; G.k41 = C.c40 * i01 + C.c41 * i11;
    // written as chains of multiply-adds (one rounding per term)
    p[0] = p[0] + G.k00 * r0 + G.k01 * r1;
    p[1] = p[1] + G.k10 * r0 + G.k11 * r1;
    p[2] = p[2] + G.k20 * r0 + G.k21 * r1;
    p[3] = p[3] + G.k30 * r0 + G.k31 * r1;
    p[4] = p[4] + G.k40 * r0 + G.k41 * r1;
    G.r00 = C.c00; G.r01 = C.c10; G.r02 = C.c20; G.r03 = C.c30; G.r04 = C.c40;
    G.r11 = C.c11; G.r12 = C.c21; G.r13 = C.c31; G.r14 = C.c41;
    const R chi = r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1);
    return pd ? chi : (R)-1;
}

// C -= K H C (a zero Gain leaves C exactly unchanged)
template <class R>
__host__ __device__ inline void kalman_cov(SymT<R> &C, const Gain<R> &G) {
    C.c00 = C.c00 - G.k00 * G.r00 - G.k01 * G.r01;
    C.c10 = C.c10 - G.k10 * G.r00 - G.k11 * G.r01;
    C.c11 = C.c11 - G.k10 * G.r01 - G.k11 * G.r11;
    C.c20 = C.c20 - G.k20 * G.r00 - G.k21 * G.r01;
    C.c21 = C.c21 - G.k20 * G.r01 - G.k21 * G.r11;
    C.c22 = C.c22 - G.k20 * G.r02 - G.k21 * G.r12;
    C.c30 = C.c30 - G.k30 * G.r00 - G.k31 * G.r01;
    C.c31 = C.c31 - G.k30 * G.r01 - G.k31 * G.r11;
    C.c32 = C.c32 - G.k30 * G.r02 - G.k31 * G.r12;
    C.c33 = C.c33 - G.k30 * G.r03 - G.k31 * G.r13;
    C.c40 = C.c40 - G.k40 * G.r00 - G.k41 * G.r01;
    C.c41 = C.c41 - G.k40 * G.r01 - G.k41 * G.r11;
    C.c42 = C.c42 - G.k40 * G.r02 - G.k41 * G.r12;
    C.c43 = C.c43 - G.k40 * G.r03 - G.k41 * G.r13;
    C.c44 = C.c44 - G.k40 * G.r04 - G.k41 * G.r14;
}

template <class R>
__host__ __device__ inline R kalman_update(R p[5], SymT<R> &C, R my, R mz, R vy, R vz) {
    Gain<R> G;
    const R chi = kalman_gain(p, C, my, mz, vy, vz, G);
    kalman_cov(C, G);
    return chi;
}

// Exact circle through C (innermost), B, A (outermost): state at A, computed
// in precision R.  Returns false if the points are degenerate or the
// direction at A is not towards +x with |sin phi| < max_sin.
template <class R, class K = float>
__host__ __device__ inline bool helix_start(R xa, R ya, R za, R xb, R yb, R xc, R yc, R zc,
                                            K kbz, float max_sin, R p[5]) {
    const R bcx = xb - xc, bcy = yb - yc;
    const R abx = xa - xb, aby = ya - yb;
    const R acx = xa - xc, acy = ya - yc;
    const R lbc = sqrt(bcx * bcx + bcy * bcy);
    const R lab = sqrt(abx * abx + aby * aby);
    const R lac = sqrt(acx * acx + acy * acy);
    const R prod = lbc * lab * lac;
    const R cross = bcx * aby - bcy * abx;
    if (!(prod > (R)0)) return false;
    const R kap = (R)2 * cross / prod;
    const R ua = (R)0.5 * kap * lab, uc = (R)0.5 * kap * lac;
    if (!(fabs(ua) < (R)1) || !(fabs(uc) < (R)1)) return false;
    // direction at A: chord angle plus half the turning angle over B -> A
    const R phia = atan2(aby, abx) + asin(ua);
    const R sn = sin(phia), cs = cos(phia);
    if (!(cs > (R)0) || !(fabs(sn) < (R)max_sin)) return false;
    p[0] = ya;
    p[1] = za;
    p[2] = sn;
    p[3] = (za - zc) / (lac * asin_over_r(uc));
    p[4] = kap / (R)kbz;          // w = -kappa / (c Bz) = kappa / kbz
    return true;
}

// ---------------------------------------------------------------------------
// Adjoint (reverse mode), written out by hand.  A symmetric matrix argument
// has a symmetric adjoint Mbar with dL = <Mbar, dM> for symmetric dM.

// Adds d<Fbar, F(p)>/dp into pbar[2..4]: the dependence of the step Jacobian
// on (s, t, w) of the state the step starts from (single precision).
__host__ __device__ inline void helix_jac_adjoint(float s, float t, float w, float dx, float kbz,
                                                  float G02, float G04, float G12, float G13,
                                                  float G14, float &bs, float &bt, float &bw) {
    const float kap = kbz * w;
    const float s2 = s + kap * dx;
    const float c1 = sqrtf((1.0f - s) * (1.0f + s));
    const float c2 = sqrtf((1.0f - s2) * (1.0f + s2));
    const float den = c1 + c2;
    const float iden = 1.0f / den;
    const float A1 = s + s2;
    const float T = A1 * iden;
    const float adx = fabsf(dx);
    const float sq = sqrtf(1.0f + T * T);
    const float chord = adx * sq;
    const float u = 0.5f * kap * chord;
    const float g = asin_over(u);
    const float gp = asin_over_d(u);
    const float gpp = asin_over_dd(u);
    const float sgn = dx >= 0.0f ? 1.0f : -1.0f;
    const float iden2 = iden * iden;
    const float N1 = den + A1 * s / c1;
    const float N2 = den + A1 * s2 / c2;
    const float dT_ds = (N1 + N2) * iden2;
    const float dT_dw = N2 * iden2 * dx * kbz;
    const float w1 = 1.0f / sqrtf((1.0f - u) * (1.0f + u));
    const float darc_dkap = sgn * 0.5f * chord * chord * gp;
    const float dchord_dT = adx * T / sq;
    const float q = sgn * w1 * dchord_dT;
    // reverse sweep
    const float b_dTds = G02 * dx + G12 * t * q;
    const float b_dTdw = G04 * dx + G14 * t * q;
    const float b_t = G12 * q * dT_ds + G14 * (q * dT_dw + darc_dkap * kbz);
    const float b_q = G12 * t * dT_ds + G14 * t * dT_dw;
    const float b_arc = G13;
    const float b_darc_dkap = G14 * t * kbz;
    const float b_N2 = (b_dTdw * dx * kbz + b_dTds) * iden2;
    const float b_N1 = b_dTds * iden2;
    const float b_w1 = b_q * sgn * dchord_dT;
    const float b_dchord_dT = b_q * sgn * w1;
    float b_T = b_dchord_dT * adx / sq;
    float b_sq = -b_dchord_dT * adx * T / (sq * sq);
    float b_chord = b_darc_dkap * sgn * chord * gp + b_arc * sgn * g;
    const float b_gp = b_darc_dkap * sgn * 0.5f * chord * chord;
    const float b_g = b_arc * sgn * chord;
    const float b_u = b_gp * gpp + b_w1 * u * w1 * w1 * w1 + b_g * gp;
    float b_kap = b_u * 0.5f * chord;
    b_chord += b_u * 0.5f * kap;
    b_sq += b_chord * adx;
    b_T += b_sq * T / sq;
    const float b_iden2 = b_dTds * N1 + (b_dTdw * dx * kbz + b_dTds) * N2;
    float b_den = b_N1 + b_N2;
    float b_A1 = b_N1 * s / c1 + b_N2 * s2 / c2;
    float b_s = b_N1 * A1 / c1;
    float b_s2 = b_N2 * A1 / c2;
    float b_c1 = -b_N1 * A1 * s / (c1 * c1);
    float b_c2 = -b_N2 * A1 * s2 / (c2 * c2);
    float b_iden = b_iden2 * 2.0f * iden;
    b_A1 += b_T * iden;
    b_iden += b_T * A1;
    b_den += -b_iden * iden * iden;
    b_c1 += b_den;
    b_c2 += b_den;
    b_s2 += -b_c2 * s2 / c2;
    b_s += -b_c1 * s / c1;
    b_s += b_A1;
    b_s2 += b_A1;
    b_s += b_s2;
    b_kap += b_s2 * dx;
    bs = b_s;
    bt = b_t;
    bw = b_kap * kbz;
}

// Reverse of one filter step (propagate by dx, then update with (my, mz)).
// In: the state (pb, Cb) the step started from, the adjoints (pbar, Cbar)
// of its result, chibar = dL/dchi2.  Out: pbar, Cbar become the adjoints of
// (pb, Cb); (mby, mbz) receive dL/d(my, mz).
template <class R>
__host__ __device__ inline void step_adjoint(const R pb[5], const SymT<R> &Cb, float dx, float kbz,
                                             R my, R mz, R vy, R vz, R chibar, R pbar[5],
                                             SymT<R> &Cbar, R &mby, R &mbz) {
    // recompute the step
    R pp[5] = {pb[0], pb[1], pb[2], pb[3], pb[4]};
    StepJac J;
    helix_step(pp, dx, kbz, 2.0f, J);
    SymT<R> P = Cb;
    sym_transport<R, false>(P, J);
    const R r0 = my - pp[0], r1 = mz - pp[1];
    const R S00 = P.c00 + vy, S01 = P.c10, S11 = P.c11 + vz;
    const R idet = (R)1 / (S00 * S11 - S01 * S01);
    const R i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
    const R a0 = i00 * r0 + i01 * r1, a1 = i01 * r0 + i11 * r1;        // a = S^-1 r
    // columns of B = P[:, 0:2]
    const R B0[5] = {P.c00, P.c10, P.c20, P.c30, P.c40};
    const R B1[5] = {P.c10, P.c11, P.c21, P.c31, P.c41};
    const R Cb_[25] = {Cbar.c00, Cbar.c10, Cbar.c20, Cbar.c30, Cbar.c40,
                       Cbar.c10, Cbar.c11, Cbar.c21, Cbar.c31, Cbar.c41,
                       Cbar.c20, Cbar.c21, Cbar.c22, Cbar.c32, Cbar.c42,
                       Cbar.c30, Cbar.c31, Cbar.c32, Cbar.c33, Cbar.c43,
                       Cbar.c40, Cbar.c41, Cbar.c42, Cbar.c43, Cbar.c44};
    R ab0 = 0, ab1 = 0;                 // abar = B^T pbar
    R CB0[5], CB1[5];                   // Cbar B
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        ab0 += B0[i] * pbar[i];
        ab1 += B1[i] * pbar[i];
        R x0 = 0, x1 = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            x0 += Cb_[i * 5 + k] * B0[k];
            x1 += Cb_[i * 5 + k] * B1[k];
        }
        CB0[i] = x0;
        CB1[i] = x1;
    }
    R BCB00 = 0, BCB01 = 0, BCB11 = 0;  // B^T Cbar B (symmetric)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        BCB00 += B0[k] * CB0[k];
        BCB01 += B0[k] * CB1[k];
        BCB11 += B1[k] * CB1[k];
    }
    // Sibar = chibar r r^T + abar r^T - B^T Cbar B
    const R Sb00 = chibar * r0 * r0 + ab0 * r0 - BCB00;
    const R Sb01 = chibar * r0 * r1 + ab0 * r1 - BCB01;
    const R Sb10 = chibar * r1 * r0 + ab1 * r0 - BCB01;
    const R Sb11 = chibar * r1 * r1 + ab1 * r1 - BCB11;
    // Sbar = -Si Sibar Si, symmetrised
    const R t00 = i00 * Sb00 + i01 * Sb10, t01 = i00 * Sb01 + i01 * Sb11;
    const R t10 = i01 * Sb00 + i11 * Sb10, t11 = i01 * Sb01 + i11 * Sb11;
    const R Sbar00 = -(t00 * i00 + t01 * i01);
    const R Sbar01 = -(R)0.5 * ((t00 * i01 + t01 * i11) + (t10 * i00 + t11 * i01));
    const R Sbar11 = -(t10 * i01 + t11 * i11);
    // rbar = 2 chibar a + Si abar
    const R rb0 = (R)2 * chibar * a0 + i00 * ab0 + i01 * ab1;
    const R rb1 = (R)2 * chibar * a1 + i01 * ab0 + i11 * ab1;
    mby = rb0;
    mbz = rb1;
    // Bbar = pbar a^T - 2 Cbar B Si
    R Bb0[5], Bb1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Bb0[i] = pbar[i] * a0 - (R)2 * (CB0[i] * i00 + CB1[i] * i01);
        Bb1[i] = pbar[i] * a1 - (R)2 * (CB0[i] * i01 + CB1[i] * i11);
    }
    // Pbar = Cbar + sym(Bbar in columns 0, 1) + Sbar in the 2x2 block
    SymT<R> Pb = Cbar;
    Pb.c00 += Bb0[0] + Sbar00;
    Pb.c10 += (R)0.5 * (Bb0[1] + Bb1[0]) + Sbar01;
    Pb.c11 += Bb1[1] + Sbar11;
    Pb.c20 += (R)0.5 * Bb0[2];
    Pb.c21 += (R)0.5 * Bb1[2];
    Pb.c30 += (R)0.5 * Bb0[3];
    Pb.c31 += (R)0.5 * Bb1[3];
    Pb.c40 += (R)0.5 * Bb0[4];
    Pb.c41 += (R)0.5 * Bb1[4];
    // adjoint of the propagated state: pbar - H^T rbar
    const R q0 = pbar[0] - rb0, q1 = pbar[1] - rb1, q2 = pbar[2], q3 = pbar[3], q4 = pbar[4];
    // Fbar = 2 Pbar F Cb, entries (0,2) (0,4) (1,2) (1,3) (1,4).  Rows 0, 1 of
    // Pbar F: column j of F adds the columns listed in sym_transport.
    const R PF00 = Pb.c00, PF01 = Pb.c10;
    const R PF02 = Pb.c20 + (R)J.f02 * Pb.c00 + (R)J.f12 * Pb.c10;
    const R PF03 = Pb.c30 + (R)J.f13 * Pb.c10;
    const R PF04 = Pb.c40 + (R)J.f04 * Pb.c00 + (R)J.f14 * Pb.c10 + (R)J.f24 * Pb.c20;
    const R PF10 = Pb.c10, PF11 = Pb.c11;
    const R PF12 = Pb.c21 + (R)J.f02 * Pb.c10 + (R)J.f12 * Pb.c11;
    const R PF13 = Pb.c31 + (R)J.f13 * Pb.c11;
    const R PF14 = Pb.c41 + (R)J.f04 * Pb.c10 + (R)J.f14 * Pb.c11 + (R)J.f24 * Pb.c21;
    const R Cc2[5] = {Cb.c20, Cb.c21, Cb.c22, Cb.c32, Cb.c42};     // column 2 of Cb
    const R Cc3[5] = {Cb.c30, Cb.c31, Cb.c32, Cb.c33, Cb.c43};
    const R Cc4[5] = {Cb.c40, Cb.c41, Cb.c42, Cb.c43, Cb.c44};
    const R r0v[5] = {PF00, PF01, PF02, PF03, PF04};
    const R r1v[5] = {PF10, PF11, PF12, PF13, PF14};
    R G02 = 0, G04 = 0, G12 = 0, G13 = 0, G14 = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        G02 += r0v[k] * Cc2[k];
        G04 += r0v[k] * Cc4[k];
        G12 += r1v[k] * Cc2[k];
        G13 += r1v[k] * Cc3[k];
        G14 += r1v[k] * Cc4[k];
    }
    // Cbar_b = F^T Pbar F
    Cbar = Pb;
    sym_transport<R, true>(Cbar, J);
    // pbar_b = F^T q + second-order term of the Jacobian
    float bs, bt, bw;
    helix_jac_adjoint((float)pb[2], (float)pb[3], (float)pb[4], dx, kbz, (float)(2 * G02),
                      (float)(2 * G04), (float)(2 * G12), (float)(2 * G13), (float)(2 * G14),
                      bs, bt, bw);
    pbar[0] = q0;
    pbar[1] = q1;
    pbar[2] = q2 + (R)J.f02 * q0 + (R)J.f12 * q1 + (R)bs;
    pbar[3] = q3 + (R)J.f13 * q1 + (R)bt;
    pbar[4] = q4 + (R)J.f04 * q0 + (R)J.f14 * q1 + (R)J.f24 * q2 + (R)bw;
}

// Reverse of helix_start: adjoint of the start state -> adjoints of the
// measurements of A (outermost), B and C (innermost).
template <class R>
__host__ __device__ inline void start_adjoint(R xa, R ya, R za, R xb, R yb, R xc, R yc, R zc,
                                              float kbz, const R pbar[5], R &bya, R &bza, R &byb,
                                              R &byc, R &bzc) {
    const R bcx = xb - xc, bcy = yb - yc;
    const R abx = xa - xb, aby = ya - yb;
    const R acx = xa - xc, acy = ya - yc;
    const R lbc = sqrt(bcx * bcx + bcy * bcy);
    const R lab = sqrt(abx * abx + aby * aby);
    const R lac = sqrt(acx * acx + acy * acy);
    const R prod = lbc * lab * lac;
    const R cross = bcx * aby - bcy * abx;
    const R kap = (R)2 * cross / prod;
    const R ua = (R)0.5 * kap * lab, uc = (R)0.5 * kap * lac;
    const R phia = atan2(aby, abx) + asin(ua);
    const R guc = asin_over_r(uc);
    const R D = lac * guc;
    const R t = (za - zc) / D;
    const R bphi = pbar[2] * cos(phia);
    const R lab2 = lab * lab;
    R b_aby = bphi * abx / lab2;
    const R b_ua = bphi / sqrt(((R)1 - ua) * ((R)1 + ua));
    bya = pbar[0];
    bza = pbar[1] + pbar[3] / D;
    bzc = -pbar[3] / D;
    const R b_D = -pbar[3] * t / D;
    R b_lac = b_D * guc;
    // d(asin(u)/u)/du
    R gp;
    if (fabs(uc) < (R)0.05) {
        const R u2 = uc * uc;
        gp = uc * ((R)1 / 3 + u2 * ((R)3 / 10 + u2 * ((R)15 / 56 + u2 * ((R)35 / 144))));
    } else {
        gp = (uc / sqrt(((R)1 - uc) * ((R)1 + uc)) - asin(uc)) / (uc * uc);
    }
    const R b_uc = b_D * lac * gp;
    const R b_kap = pbar[4] / (R)kbz + b_ua * (R)0.5 * lab + b_uc * (R)0.5 * lac;
    R b_lab = b_ua * (R)0.5 * kap;
    b_lac += b_uc * (R)0.5 * kap;
    const R b_cross = (R)2 * b_kap / prod;
    const R b_prod = -b_kap * kap / prod;
    const R b_lbc = b_prod * lab * lac;
    b_lab += b_prod * lbc * lac;
    b_lac += b_prod * lbc * lab;
    b_aby += b_cross * bcx;
    R b_bcy = -b_cross * abx;
    b_bcy += b_lbc * bcy / lbc;
    b_aby += b_lab * aby / lab;
    const R b_acy = b_lac * acy / lac;
    (void)acx;
    byb = b_bcy - b_aby;
    byc = -b_bcy - b_acy;
    bya += b_aby + b_acy;
}
