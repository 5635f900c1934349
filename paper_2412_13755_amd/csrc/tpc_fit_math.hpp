// Single-precision helix-fit arithmetic shared by the forward fit and its
// adjoint.  State p = (y, z, s = sin phi, t = tan lambda, w = q/pT) on a
// pad-row plane x, track oriented towards +x, curvature kappa = -c Bz w
// (counter-clockwise positive).  Covariance in registers as the 15 entries
// of its lower triangle.  No MFMA: a 5x5 symmetric update is not a dense
// contraction worth a matrix core; everything is plain VALU work.
#pragma once

#include <hip/hip_runtime.h>

#define TPC_C_LIGHT 0.00299792458f

struct Sym5 {
    // lower triangle, row by row: 00 10 11 20 21 22 30 31 32 33 40 41 42 43 44
    float c00, c10, c11, c20, c21, c22, c30, c31, c32, c33, c40, c41, c42, c43, c44;
};

__host__ __device__ inline float asin_over(float u) {
    // asin(u)/u with its Taylor series near 0 (terms to u^8)
    if (fabsf(u) < 0.05f) {
        float u2 = u * u;
        return 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f + u2 * (35.0f / 1152.0f))));
    }
    return asinf(u) / u;
}

// derivative of asin(u)/u
__host__ __device__ inline float asin_over_d(float u) {
    if (fabsf(u) < 0.05f) {
        float u2 = u * u;
        return u * (1.0f / 3.0f + u2 * (3.0f / 10.0f + u2 * (15.0f / 56.0f + u2 * (35.0f / 144.0f))));
    }
    return (u / sqrtf(1.0f - u * u) - asinf(u)) / (u * u);
}

// Jacobian entries that differ from the identity.
struct StepJac {
    float f02, f04, f12, f13, f14, f24;
};

// Exact helix step from x to x + dx.  Returns false when |sin phi| reaches
// max_sin (then p is left unchanged).
__host__ __device__ inline bool helix_step(float p[5], float dx, float kbz, float max_sin,
                                           StepJac &J) {
    // kbz = -c Bz: kappa = kbz * w
    const float s = p[2], t = p[3], w = p[4];
    const float kap = kbz * w;
    const float s2 = s + kap * dx;
    if (!(fabsf(s) < max_sin) || !(fabsf(s2) < max_sin)) return false;
    const float c1 = sqrtf((1.0f - s) * (1.0f + s));
    const float c2 = sqrtf((1.0f - s2) * (1.0f + s2));
    const float den = c1 + c2;
    const float iden = 1.0f / den;
    const float T = (s + s2) * iden;
    const float adx = fabsf(dx);
    const float sq = sqrtf(1.0f + T * T);
    const float chord = adx * sq;
    const float u = 0.5f * kap * chord;
    const float g = asin_over(u);
    const float sgn = dx >= 0.0f ? 1.0f : -1.0f;
    const float arc = sgn * chord * g;
    // Jacobian
    const float iden2 = iden * iden;
    const float dTs_p = (den + (s + s2) * s / c1) * iden2;
    const float dTs2_p = (den + (s + s2) * s2 / c2) * iden2;
    const float dT_ds = dTs_p + dTs2_p;
    const float dT_dw = dTs2_p * dx * kbz;
    const float darc_dchord = sgn / sqrtf((1.0f - u) * (1.0f + u));
    const float darc_dkap = sgn * 0.5f * chord * chord * asin_over_d(u);
    const float dchord_dT = adx * T / sq;
    const float q = darc_dchord * dchord_dT;
    J.f02 = dx * dT_ds;
    J.f04 = dx * dT_dw;
    J.f12 = t * q * dT_ds;
    J.f13 = arc;
    J.f14 = t * (q * dT_dw + darc_dkap * kbz);
    J.f24 = dx * kbz;
    p[0] += dx * T;
    p[1] += t * arc;
    p[2] = s2;
    return true;
}

// C <- F C F^T for the sparse step Jacobian.
__host__ __device__ inline void cov_step(Sym5 &C, const StepJac &J) {
    // A = F C (full 5x5 rows 0..2; rows 3, 4 are those of C)
    const float C00 = C.c00, C01 = C.c10, C02 = C.c20, C03 = C.c30, C04 = C.c40;
    const float C11 = C.c11, C12 = C.c21, C13 = C.c31, C14 = C.c41;
    const float C22 = C.c22, C23 = C.c32, C24 = C.c42;
    const float C33 = C.c33, C34 = C.c43, C44 = C.c44;
    // row 0 of A
    const float A00 = C00 + J.f02 * C02 + J.f04 * C04;
    const float A01 = C01 + J.f02 * C12 + J.f04 * C14;
    const float A02 = C02 + J.f02 * C22 + J.f04 * C24;
    const float A03 = C03 + J.f02 * C23 + J.f04 * C34;
    const float A04 = C04 + J.f02 * C24 + J.f04 * C44;
    // row 1
    const float A10 = C01 + J.f12 * C02 + J.f13 * C03 + J.f14 * C04;
    const float A11 = C11 + J.f12 * C12 + J.f13 * C13 + J.f14 * C14;
    const float A12 = C12 + J.f12 * C22 + J.f13 * C23 + J.f14 * C24;
    const float A13 = C13 + J.f12 * C23 + J.f13 * C33 + J.f14 * C34;
    const float A14 = C14 + J.f12 * C24 + J.f13 * C34 + J.f14 * C44;
    // row 2
    const float A20 = C02 + J.f24 * C04;
    const float A21 = C12 + J.f24 * C14;
    const float A22 = C22 + J.f24 * C24;
    const float A23 = C23 + J.f24 * C34;
    const float A24 = C24 + J.f24 * C44;
    // C' = A F^T, lower triangle
    C.c00 = A00 + J.f02 * A02 + J.f04 * A04;
    C.c10 = A10 + J.f02 * A12 + J.f04 * A14;
    C.c11 = A11 + J.f12 * A12 + J.f13 * A13 + J.f14 * A14;
    C.c20 = A20 + J.f02 * A22 + J.f04 * A24;
    C.c21 = A21 + J.f12 * A22 + J.f13 * A23 + J.f14 * A24;
    C.c22 = A22 + J.f24 * A24;
    C.c30 = C03 + J.f02 * C23 + J.f04 * C34;     // row 3 of A is row 3 of C
    C.c31 = C13 + J.f12 * C23 + J.f13 * C33 + J.f14 * C34;
    C.c32 = C23 + J.f24 * C34;
    C.c33 = C33;
    C.c40 = C04 + J.f02 * C24 + J.f04 * C44;
    C.c41 = C14 + J.f12 * C24 + J.f13 * C34 + J.f14 * C44;
    C.c42 = C24 + J.f24 * C44;
    C.c43 = C34;
    C.c44 = C44;
}

// Kalman update with measurement (my, mz); returns the chi2 increment, or a
// negative value if the residual covariance is not positive definite.
__host__ __device__ inline float kalman_update(float p[5], Sym5 &C, float my, float mz, float vy,
                                               float vz) {
    const float r0 = my - p[0], r1 = mz - p[1];
    const float S00 = C.c00 + vy, S01 = C.c10, S11 = C.c11 + vz;
    const float det = S00 * S11 - S01 * S01;
    if (!(det > 0.0f)) return -1.0f;
    const float idet = 1.0f / det;
    const float i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
    // K = C[:, 0:2] S^-1 ; columns of C: (c_i0, c_i1)
    const float k00 = C.c00 * i00 + C.c10 * i01, k01 = C.c00 * i01 + C.c10 * i11;
    const float k10 = C.c10 * i00 + C.c11 * i01, k11 = C.c10 * i01 + C.c11 * i11;
    const float k20 = C.c20 * i00 + C.c21 * i01, k21 = C.c20 * i01 + C.c21 * i11;
    const float k30 = C.c30 * i00 + C.c31 * i01, k31 = C.c30 * i01 + C.c31 * i11;
    const float k40 = C.c40 * i00 + C.c41 * i01, k41 = C.c40 * i01 + C.c41 * i11;
    p[0] += k00 * r0 + k01 * r1;
    p[1] += k10 * r0 + k11 * r1;
    p[2] += k20 * r0 + k21 * r1;
    p[3] += k30 * r0 + k31 * r1;
    p[4] += k40 * r0 + k41 * r1;
    // C -= K (rows 0, 1 of C)
    const float r00 = C.c00, r01 = C.c10, r02 = C.c20, r03 = C.c30, r04 = C.c40;
    const float r11 = C.c11, r12 = C.c21, r13 = C.c31, r14 = C.c41;
    C.c00 -= k00 * r00 + k01 * r01;
    C.c10 -= k10 * r00 + k11 * r01;
    C.c11 -= k10 * r01 + k11 * r11;
    C.c20 -= k20 * r00 + k21 * r01;
    C.c21 -= k20 * r01 + k21 * r11;
    C.c22 -= k20 * r02 + k21 * r12;
    C.c30 -= k30 * r00 + k31 * r01;
    C.c31 -= k30 * r01 + k31 * r11;
    C.c32 -= k30 * r02 + k31 * r12;
    C.c33 -= k30 * r03 + k31 * r13;
    C.c40 -= k40 * r00 + k41 * r01;
    C.c41 -= k40 * r01 + k41 * r11;
    C.c42 -= k40 * r02 + k41 * r12;
    C.c43 -= k40 * r03 + k41 * r13;
    C.c44 -= k40 * r04 + k41 * r14;
    return r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1);
}

// Exact circle through C (innermost), B, A (outermost): state at A.
// Returns false if the three points are degenerate or the direction at A is
// not towards +x with |sin phi| < max_sin.
__host__ __device__ inline bool helix_start(float xa, float ya, float za, float xb, float yb,
                                            float xc, float yc, float zc, float kbz,
                                            float max_sin, float p[5]) {
    const float bcx = xb - xc, bcy = yb - yc;
    const float abx = xa - xb, aby = ya - yb;
    const float acx = xa - xc, acy = ya - yc;
    const float lbc = sqrtf(bcx * bcx + bcy * bcy);
    const float lab = sqrtf(abx * abx + aby * aby);
    const float lac = sqrtf(acx * acx + acy * acy);
    const float prod = lbc * lab * lac;
    const float cross = bcx * aby - bcy * abx;
    if (!(prod > 0.0f)) return false;
    const float kap = 2.0f * cross / prod;
    const float ua = 0.5f * kap * lab, uc = 0.5f * kap * lac;
    if (!(fabsf(ua) < 1.0f) || !(fabsf(uc) < 1.0f)) return false;
    // direction at A: chord angle plus half the turning angle over A-B
    const float phia = atan2f(aby, abx) + asinf(ua);
    float sn, cs;
    sincosf(phia, &sn, &cs);
    if (!(cs > 0.0f) || !(fabsf(sn) < max_sin)) return false;
    p[0] = ya;
    p[1] = za;
    p[2] = sn;
    p[3] = (za - zc) / (lac * asin_over(uc));
    p[4] = kap / kbz;          // w = -kappa / (c Bz) = kappa / kbz
    return true;
}
