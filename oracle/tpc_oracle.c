/*
 * CPU oracle for TPC track reconstruction: neighbour finding, cellular
 * automaton seeding and a Kalman helix fit.  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the CPU baseline leg of the benchmark call it;
 * the GPU library never does, and the two share no code.
 *
 * The paper (Sec. 4.2 and Sec. 5) states that TPC track reconstruction is the
 * work that fully loads the farm's GPUs, but it does not describe the
 * algorithm.  Every step below is therefore a textbook reading, written as
 * plainly as possible:
 *
 *   neighbours      windowed triplet search with a second-difference score;
 *                   single precision, every operation rounded (no FMA), so a
 *                   GPU implementation can match it bit for bit
 *   ca_seed         mutual links -> maximal chains -> end claims -> seeds
 *   fit             exact three-point helix start + extended Kalman filter
 *                   through the hits inwards, double precision throughout
 *   neighbours_skip partners up to two rows away where adjacent rows give none
 *   fit_rows        the fit over seeds that skip rows, per-cluster errors
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "tpc_oracle.h"

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Neighbours.  For every cluster h of pad row r (1 <= r <= R-2) of every     */
/* (frame, sector), choose the pair (d in row r-1, u in row r+1) that passes  */
/* the position windows and the second-difference cuts and minimises          */
/*   q = (dy*dy + dz*dz),  dy = (y_u - y_h) - (y_h - y_d),  dz likewise,      */
/* ties broken by the smaller u id, then the smaller d id.  Rows 0 and R-1    */
/* get no partners.  A non-finite coordinate fails every comparison.          */
/* ------------------------------------------------------------------------ */
void oracle_neighbours(int32_t n_segments, int32_t n_rows, const int32_t *row_offsets,
                       const float *y, const float *z, float win_y, float win_z,
                       float cut_y, float cut_z, int32_t *up, int32_t *dn)
{
    int32_t n = row_offsets[n_segments];
    for (int32_t i = 0; i < n; ++i) { up[i] = -1; dn[i] = -1; }

    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t seg = 0; seg < n_segments; ++seg) {
        int32_t r = seg % n_rows;
        if (r == 0 || r == n_rows - 1) continue;
        int32_t h0 = row_offsets[seg], h1 = row_offsets[seg + 1];
        int32_t u0 = row_offsets[seg + 1], u1 = row_offsets[seg + 2];   /* row r+1 */
        int32_t d0 = row_offsets[seg - 1], d1 = row_offsets[seg];       /* row r-1 */
        /* the down clusters inside h's window, in ascending id: the window   */
        /* test of d does not depend on u, so it is made once per h and the   */
        /* pair loop below visits the same d, in the same order, as a test    */
        /* repeated for every u would                                         */
        int32_t *dl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d1 - d0 + 1));
        float *dby = (float *)malloc(sizeof(float) * (size_t)(d1 - d0 + 1));
        float *dbz = (float *)malloc(sizeof(float) * (size_t)(d1 - d0 + 1));
        for (int32_t h = h0; h < h1; ++h) {
            int found = 0;
            float best_q = 0.0f;
            int32_t best_u = -1, best_d = -1;
            int32_t nd = 0;
            for (int32_t d = d0; d < d1; ++d) {
                float by = y[h] - y[d];
                float bz = z[h] - z[d];
                if (!(fabsf(by) <= win_y && fabsf(bz) <= win_z)) continue;
                dl[nd] = d; dby[nd] = by; dbz[nd] = bz; ++nd;
            }
            for (int32_t u = u0; u < u1; ++u) {
                float ay = y[u] - y[h];
                float az = z[u] - z[h];
                if (!(fabsf(ay) <= win_y && fabsf(az) <= win_z)) continue;
                for (int32_t k = 0; k < nd; ++k) {
                    int32_t d = dl[k];
                    float by = dby[k];
                    float bz = dbz[k];
                    float dy = ay - by;
                    float dz = az - bz;
                    if (!(fabsf(dy) <= cut_y && fabsf(dz) <= cut_z)) continue;
                    float qy = dy * dy;
                    float qz = dz * dz;
                    float q = qy + qz;
                    /* u and d ascend, so strict '<' keeps the smallest (q, u, d) */
                    if (!found || q < best_q) {
                        found = 1; best_q = q; best_u = u; best_d = d;
                    }
                }
            }
            up[h] = best_u;
            dn[h] = best_d;
        }
        free(dl); free(dby); free(dbz);
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbours across a missing pad row.  The partners of h (row r, 1 <= r <=  */
/* R-2) may lie one or two rows away: d in row r-a, u in row r+b, a and b in  */
/* {1, 2}, both rows inside the sector.  With A = y_u - y_h, B = y_h - y_d    */
/* (z likewise) a triplet passes if                                           */
/*   |A| <= b win, |B| <= a win (y and z with their windows) and              */
/*   |D| <= cut,  D = g (A/b - B/a),  g = 2/(a+b):                            */
/* D is the divided second difference scaled to unit row pitch -- zero on a   */
/* straight line, and on a parabola the same value for every (a, b) -- and    */
/* at a = b = 1 it is the adjacent-row dy above.  A triplet that spans fewer  */
/* rows always wins (a+b = 2, then 3, then 4), so h keeps its adjacent-row    */
/* result whenever it has one.  Within a span: smallest q = Dy^2 + Dz^2, then */
/* smaller u id, then smaller d id.  Single precision, one rounding per       */
/* operation: b win, A/b and B/a are exact (a, b powers of two) and g is      */
/* 2/(a+b) rounded once.                                                      */
/* ------------------------------------------------------------------------ */
void oracle_neighbours_skip(int32_t n_segments, int32_t n_rows, const int32_t *row_offsets,
                            const float *y, const float *z, float win_y, float win_z,
                            float cut_y, float cut_z, int32_t *up, int32_t *dn)
{
    int32_t n = row_offsets[n_segments];
    for (int32_t i = 0; i < n; ++i) { up[i] = -1; dn[i] = -1; }

    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t seg = 0; seg < n_segments; ++seg) {
        int32_t r = seg % n_rows;
        if (r == 0 || r == n_rows - 1) continue;
        for (int32_t h = row_offsets[seg]; h < row_offsets[seg + 1]; ++h) {
            int found = 0;
            float best_q = 0.0f;
            int32_t best_u = -1, best_d = -1;
            for (int span = 2; span <= 4 && !found; ++span) {
                for (int a = 1; a <= 2; ++a) {
                    int b = span - a;
                    if (b < 1 || b > 2 || r - a < 0 || r + b > n_rows - 1) continue;
                    float fa = (float)a, fb = (float)b;
                    float g = 2.0f / (float)span;
                    int32_t su = seg + b, sd = seg - a;
                    for (int32_t u = row_offsets[su]; u < row_offsets[su + 1]; ++u) {
                        float Ay = y[u] - y[h];
                        float Az = z[u] - z[h];
                        if (!(fabsf(Ay) <= fb * win_y && fabsf(Az) <= fb * win_z)) continue;
                        for (int32_t d = row_offsets[sd]; d < row_offsets[sd + 1]; ++d) {
                            float By = y[h] - y[d];
                            float Bz = z[h] - z[d];
                            if (!(fabsf(By) <= fa * win_y && fabsf(Bz) <= fa * win_z)) continue;
                            float ty = Ay / fb, sy = By / fa;
                            float tz = Az / fb, sz = Bz / fa;
                            float ey = ty - sy, ez = tz - sz;
                            float Dy = g * ey, Dz = g * ez;
                            if (!(fabsf(Dy) <= cut_y && fabsf(Dz) <= cut_z)) continue;
                            float qy = Dy * Dy;
                            float qz = Dz * Dz;
                            float q = qy + qz;
                            int better = !found || q < best_q ||
                                         (q == best_q && (u < best_u || (u == best_u && d < best_d)));
                            if (better) { found = 1; best_q = q; best_u = u; best_d = d; }
                        }
                    }
                }
            }
            up[h] = best_u;
            dn[h] = best_d;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Seeding.                                                                   */
/*  links:  Lup[h] = up[h] if dn[up[h]] == h;  Ldn[h] = dn[h] if up[dn[h]]==h */
/*  chains: from a bottom b (no Ldn, has Lup) follow Lup to the top t;        */
/*          core length m (>= 2)                                              */
/*  claims: a chain with m >= min_hits-2 claims dn[b] and up[t] if these are  */
/*          not linked; each claimed cluster goes to the smallest key         */
/*          (-m, b)                                                           */
/*  seeds:  [dn[b] if won] + core + [up[t] if won], kept if >= min_hits hits, */
/*          listed in ascending id of their first hit                         */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t first; int32_t b; int32_t len; int32_t eb; int32_t et; } seed_rec;

static int cmp_seed(const void *a, const void *b)
{
    const seed_rec *x = (const seed_rec *)a, *y = (const seed_rec *)b;
    return (x->first > y->first) - (x->first < y->first);
}

int32_t oracle_ca_seed(int32_t n_segments, int32_t n_sectors, int32_t n_rows,
                       const int32_t *row_offsets, const int32_t *up, const int32_t *dn,
                       int32_t min_hits, int32_t cap_seeds, int32_t cap_hits,
                       int32_t *n_seeds_out, int32_t *n_hits_out, int32_t *offsets,
                       int32_t *hits, int32_t *frame, int32_t *sector, int32_t *first_row)
{
    int32_t n = row_offsets[n_segments];
    int32_t *Lup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *Ldn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *seg_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t *claim = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *top = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *core = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    seed_rec *recs = (seed_rec *)malloc(sizeof(seed_rec) * (size_t)(n > 0 ? n : 1));

    for (int32_t s = 0; s < n_segments; ++s)
        for (int32_t i = row_offsets[s]; i < row_offsets[s + 1]; ++i) seg_of[i] = s;

    for (int32_t h = 0; h < n; ++h) {
        Lup[h] = (up[h] >= 0 && dn[up[h]] == h) ? up[h] : -1;
        Ldn[h] = (dn[h] >= 0 && up[dn[h]] == h) ? dn[h] : -1;
        claim[h] = UINT64_MAX;
        top[h] = -1;
        core[h] = 0;
    }
    /* chains */
    for (int32_t b = 0; b < n; ++b) {
        if (!(Ldn[b] == -1 && Lup[b] != -1)) continue;
        int32_t t = b, m = 1;
        while (Lup[t] != -1) { t = Lup[t]; ++m; }
        top[b] = t;
        core[b] = m;
    }
    /* claims */
    for (int32_t b = 0; b < n; ++b) {
        if (top[b] < 0 || core[b] < min_hits - 2) continue;
        uint64_t key = ((uint64_t)(2147483648u - (uint32_t)core[b]) << 32) | (uint32_t)b;
        int32_t ends[2] = {dn[b], up[top[b]]};
        for (int k = 0; k < 2; ++k) {
            int32_t e = ends[k];
            if (e < 0 || Lup[e] != -1 || Ldn[e] != -1) continue;
            if (key < claim[e]) claim[e] = key;
        }
    }
    /* seeds */
    int32_t ns = 0;
    for (int32_t b = 0; b < n; ++b) {
        if (top[b] < 0) continue;
        int32_t m = core[b];
        int won_b = 0, won_t = 0;
        if (m >= min_hits - 2) {
            uint64_t key = ((uint64_t)(2147483648u - (uint32_t)m) << 32) | (uint32_t)b;
            int32_t eb = dn[b], et = up[top[b]];
            won_b = (eb >= 0 && claim[eb] == key);
            won_t = (et >= 0 && claim[et] == key);
        }
        int32_t len = m + won_b + won_t;
        if (len < min_hits) continue;
        recs[ns].b = b;
        recs[ns].len = len;
        recs[ns].eb = won_b ? dn[b] : -1;
        recs[ns].et = won_t ? up[top[b]] : -1;
        recs[ns].first = won_b ? dn[b] : b;
        ++ns;
    }
    qsort(recs, (size_t)ns, sizeof(seed_rec), cmp_seed);

    int32_t nh = 0;
    for (int32_t i = 0; i < ns; ++i) nh += recs[i].len;
    *n_seeds_out = ns;
    *n_hits_out = nh;
    int32_t status = 0;
    if (ns > cap_seeds || nh > cap_hits) status = -2;
    else {
        int32_t pos = 0;
        for (int32_t i = 0; i < ns; ++i) {
            offsets[i] = pos;
            int32_t f = recs[i].first;
            int32_t seg = seg_of[f];
            frame[i] = seg / (n_sectors * n_rows);
            sector[i] = (seg / n_rows) % n_sectors;
            first_row[i] = seg % n_rows;
            if (recs[i].eb >= 0) hits[pos++] = recs[i].eb;
            for (int32_t c = recs[i].b; c != -1; c = Lup[c]) hits[pos++] = c;
            if (recs[i].et >= 0) hits[pos++] = recs[i].et;
        }
        offsets[ns] = pos;
    }
    free(Lup); free(Ldn); free(seg_of); free(claim); free(top); free(core); free(recs);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Helix propagation between pad-row planes, double precision.               */
/* State p = (y, z, s = sin phi, t = tan lambda, w = q/pT) at plane x; the    */
/* track is oriented towards +x.  Curvature kappa = -c * Bz * w (ccw > 0).    */
/* ------------------------------------------------------------------------ */
#define C_LIGHT 0.00299792458

/* g(u) = asin(u)/u, g(0) = 1 */
static double g_of(double u)
{
    if (fabs(u) < 1e-2) {
        double u2 = u * u;
        return 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0)));
    }
    return asin(u) / u;
}

/* g'(u) = (u / sqrt(1-u^2) - asin(u)) / u^2 */
static double gprime_of(double u)
{
    if (fabs(u) < 1e-2) {
        double u2 = u * u;
        return u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0)));
    }
    return (u / sqrt(1.0 - u * u) - asin(u)) / (u * u);
}

/* Moves p from plane x to plane x + dx along the exact helix.  F (row-major
 * 5x5, may be NULL) receives d p_out / d p_in.  Returns 0, or 2 if the
 * direction reaches |sin phi| >= max_sin. */
int32_t oracle_propagate(const double *p, double dx, double bz, double max_sin,
                         double *pout, double *F)
{
    double y = p[0], z = p[1], s = p[2], t = p[3], w = p[4];
    double kap = -C_LIGHT * bz * w;
    double s2 = s + kap * dx;
    if (!(fabs(s) < max_sin) || !(fabs(s2) < max_sin)) return 2;
    double c1 = sqrt(1.0 - s * s);
    double c2 = sqrt(1.0 - s2 * s2);
    double den = c1 + c2;
    double T = (s + s2) / den;
    double ady = fabs(dx);
    double sgn = dx >= 0.0 ? 1.0 : -1.0;
    double chord = ady * sqrt(1.0 + T * T);
    double u = kap * chord / 2.0;
    double ds = sgn * chord * g_of(u);
    pout[0] = y + dx * T;
    pout[1] = z + t * ds;
    pout[2] = s2;
    pout[3] = t;
    pout[4] = w;
    if (F) {
        double dkap_dw = -C_LIGHT * bz;
        /* partial derivatives of T(s, s2) */
        double dT_ds_p = (den + (s + s2) * s / c1) / (den * den);
        double dT_ds2_p = (den + (s + s2) * s2 / c2) / (den * den);
        double dT_ds = dT_ds_p + dT_ds2_p;             /* ds2/ds = 1 */
        double dT_dw = dT_ds2_p * dx * dkap_dw;        /* ds2/dw = dx dkap/dw */
        /* ds = sgn * chord * g(kap * chord / 2) */
        double dds_dchord = sgn / sqrt(1.0 - u * u);   /* d(chord g(u))/dchord = g + u g' */
        double dds_dkap = sgn * chord * chord / 2.0 * gprime_of(u);
        double dchord_dT = ady * T / sqrt(1.0 + T * T);
        double dds_ds = dds_dchord * dchord_dT * dT_ds;
        double dds_dw = dds_dchord * dchord_dT * dT_dw + dds_dkap * dkap_dw;
        for (int i = 0; i < 25; ++i) F[i] = 0.0;
        for (int i = 0; i < 5; ++i) F[i * 5 + i] = 1.0;
        F[0 * 5 + 2] = dx * dT_ds;
        F[0 * 5 + 4] = dx * dT_dw;
        F[1 * 5 + 2] = t * dds_ds;
        F[1 * 5 + 3] = ds;
        F[1 * 5 + 4] = t * dds_dw;
        F[2 * 5 + 4] = dx * dkap_dw;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fit.  For each seed with hits k = 0..n-1 (ascending pad row):             */
/*  start  exact circle through hits A = n-1, B = (n-1)/2, C = 0 gives the    */
/*         curvature, the direction at A and tan lambda; state at x_A with    */
/*         y, z of A and covariance diag(sy^2, sz^2, v_s, v_t, v_w)           */
/*  filter for k = n-2 .. 0: propagate to x_k, C <- F C F^T, then update with */
/*         the measurement (y_k, z_k): r = m - (y, z), S = C_yz + diag(sy^2,  */
/*         sz^2), K = C H^T S^-1, p += K r, C -= K H C, chi2 += r^T S^-1 r    */
/*  output state and covariance at x_0, chi2, ndf = 2n - 5                    */
/* Measurements are corrected by a per (sector, row) map when one is given.   */
/* ------------------------------------------------------------------------ */
static void mat5_mul(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 5; ++k) acc += A[i * 5 + k] * B[k * 5 + j];
            C[i * 5 + j] = acc;
        }
}

/* Prediction: p, C (full 5x5) moved to the plane dx away, C <- F C F^T.
 * Returns the status of the helix step (0 or 2). */
static int32_t predict(double *p, double *C, double dx, const oracle_fit_params *prm)
{
    double pp[5], F[25], FC[25], Ft[25];
    int32_t st = oracle_propagate(p, dx, prm->bz, prm->max_sin, pp, F);
    if (st) return st;
    mat5_mul(F, C, FC);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Ft[i * 5 + j] = F[j * 5 + i];
    mat5_mul(FC, Ft, C);
    for (int i = 0; i < 5; ++i) p[i] = pp[i];
    return 0;
}

/* chi2 of the predicted residual of measurement (my, mz) against the state
 * p with covariance C; NaN if the residual covariance is not positive. */
static double resid_chi2(const double *p, const double *C, double my, double mz, double vy, double vz)
{
    double r0 = my - p[0], r1 = mz - p[1];
    double S00 = C[0] + vy, S01 = C[1], S10 = C[5], S11 = C[6] + vz;
    double det = S00 * S11 - S01 * S10;
    if (!(det > 0.0)) return NAN;
    double Si00 = S11 / det, Si01 = -S01 / det, Si10 = -S10 / det, Si11 = S00 / det;
    return r0 * (Si00 * r0 + Si01 * r1) + r1 * (Si10 * r0 + Si11 * r1);
}

/* Kalman update of the predicted p, C with the measurement (my, mz), H = [I2 0]:
 * r = m - (y, z), S = C_yz + diag(vy, vz), K = C H^T S^-1, p += K r,
 * C -= K H C.  Adds r^T S^-1 r to *chi2.  Returns 0, or 3 if S is singular
 * or the result is not finite. */
static int32_t update(double *p, double *C, double my, double mz, double vy, double vz, double *chi2)
{
    double Cp[25];
    for (int i = 0; i < 25; ++i) Cp[i] = C[i];
    double r0 = my - p[0], r1 = mz - p[1];
    double S00 = Cp[0] + vy, S01 = Cp[1], S10 = Cp[5], S11 = Cp[6] + vz;
    double det = S00 * S11 - S01 * S10;
    if (!(det > 0.0)) return 3;
    double Si00 = S11 / det, Si01 = -S01 / det, Si10 = -S10 / det, Si11 = S00 / det;
    double K[10];
    for (int i = 0; i < 5; ++i) {
        K[i * 2 + 0] = Cp[i * 5 + 0] * Si00 + Cp[i * 5 + 1] * Si10;
        K[i * 2 + 1] = Cp[i * 5 + 0] * Si01 + Cp[i * 5 + 1] * Si11;
    }
    for (int i = 0; i < 5; ++i) p[i] = p[i] + K[i * 2 + 0] * r0 + K[i * 2 + 1] * r1;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
            C[i * 5 + j] = Cp[i * 5 + j] - (K[i * 2 + 0] * Cp[0 * 5 + j] + K[i * 2 + 1] * Cp[1 * 5 + j]);
    *chi2 += r0 * (Si00 * r0 + Si01 * r1) + r1 * (Si10 * r0 + Si11 * r1);
    int finite = isfinite(*chi2);
    for (int i = 0; i < 5; ++i) finite &= isfinite(p[i]);
    return finite ? 0 : 3;
}

/* Exact circle through hits n-1 (outermost), (n-1)/2 and 0: the state at
 * x of hit n-1 and the start covariance; returns 0 or 1 (degenerate points,
 * or a direction at the start not towards +x or with |sin phi| >= max_sin).
 * With smargin non-null also the distance of the start direction from those
 * two thresholds, min(max_sin - |sin phi|, cos phi) (-inf if degenerate). */
static int32_t start_points_m(int32_t n, const double *xs, const double *ys, const double *zs,
                              const oracle_fit_params *prm, double *p, double *C, double *smargin)
{
    int a = n - 1, b = (n - 1) / 2, c = 0;
    double bcx = xs[b] - xs[c], bcy = ys[b] - ys[c];
    double abx = xs[a] - xs[b], aby = ys[a] - ys[b];
    double acx = xs[a] - xs[c], acy = ys[a] - ys[c];
    double lbc = sqrt(bcx * bcx + bcy * bcy);
    double lab = sqrt(abx * abx + aby * aby);
    double lac = sqrt(acx * acx + acy * acy);
    double cross = bcx * aby - bcy * abx;
    double prod = lbc * lab * lac;
    double kap0 = 2.0 * cross / prod;
    double ua = kap0 * lab / 2.0, uc = kap0 * lac / 2.0;
    int32_t st = 0;
    if (!(prod > 0.0) || !(fabs(ua) < 1.0) || !(fabs(uc) < 1.0)) st = 1;
    double phiA = atan2(aby, abx) + asin(st ? 0.0 : ua);
    p[0] = ys[a];
    p[1] = zs[a];
    p[2] = sin(phiA);
    p[3] = (zs[a] - zs[c]) / (lac * g_of(uc));
    p[4] = -kap0 / (C_LIGHT * prm->bz);
    if (!st && (!(cos(phiA) > 0.0) || !(fabs(p[2]) < prm->max_sin))) st = 1;
    if (smargin) {
        double m1 = prm->max_sin - fabs(p[2]), m2 = cos(phiA);
        *smargin = (!(prod > 0.0) || !(fabs(ua) < 1.0) || !(fabs(uc) < 1.0)) ? -INFINITY : (m1 < m2 ? m1 : m2);
    }
    for (int i = 0; i < 25; ++i) C[i] = 0.0;
    C[0] = prm->sigma_y * prm->sigma_y;
    C[6] = prm->sigma_z * prm->sigma_z;
    C[12] = prm->var_sin0;
    C[18] = prm->var_tgl0;
    C[24] = prm->var_qpt0;
    return st;
}

static int32_t start_points(int32_t n, const double *xs, const double *ys, const double *zs,
                            const oracle_fit_params *prm, double *p, double *C)
{
    return start_points_m(n, xs, ys, zs, prm, p, C, NULL);
}

/* Inward fit of n points at planes xs (ascending), as described above: state
 * p and full covariance C at xs[0] (or where the filter stopped), chi2, status.
 * With margin non-null also the fit's closest approach to its direction
 * thresholds: the start's (start_points_m), then max_sin - max(|s|, |s'|)
 * of every helix step taken (negative at a step that failed); only a report,
 * the fit is the same. */
static int32_t fit_points_m(int32_t n, const double *xs, const double *ys, const double *zs,
                            const oracle_fit_params *prm, double *xo, double *p, double *C, double *chi2o,
                            double *margin)
{
    *chi2o = 0.0;
    *xo = 0.0;
    for (int i = 0; i < 5; ++i) p[i] = 0.0;
    for (int i = 0; i < 25; ++i) C[i] = 0.0;
    if (margin) *margin = -INFINITY;
    if (n < 3) return 1;
    double mg = 0.0;
    int32_t st = start_points_m(n, xs, ys, zs, prm, p, C, &mg);
    int a = n - 1;
    double vy = prm->sigma_y * prm->sigma_y, vz = prm->sigma_z * prm->sigma_z;
    double chi2 = 0.0;
    double xcur = xs[a];
    for (int k = n - 2; k >= 0 && !st; --k) {
        double s1 = p[2], s2 = s1 - C_LIGHT * prm->bz * p[4] * (xs[k] - xs[k + 1]);
        double ms = prm->max_sin - (fabs(s1) > fabs(s2) ? fabs(s1) : fabs(s2));
        if (ms < mg) mg = ms;
        if (predict(p, C, xs[k] - xs[k + 1], prm)) { st = 2; break; }
        xcur = xs[k];
        if (update(p, C, ys[k], zs[k], vy, vz, &chi2)) { st = 3; break; }
    }
    *xo = xcur;
    *chi2o = chi2;
    if (margin) *margin = mg;
    return st;
}

static int32_t fit_points(int32_t n, const double *xs, const double *ys, const double *zs,
                          const oracle_fit_params *prm, double *xo, double *p, double *C, double *chi2o)
{
    return fit_points_m(n, xs, ys, zs, prm, xo, p, C, chi2o, NULL);
}

static void pack_cov(const double *C, double *co)
{
    /* packed lower triangle, row by row: (0,0) (1,0) (1,1) (2,0) ... */
    int q = 0;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) co[q++] = C[i * 5 + j];
}

static void fit_one(int32_t n, const int32_t *hit, int32_t sec, int32_t row0,
                    const double *y, const double *z, const double *row_x, int32_t n_rows,
                    const double *map, const oracle_fit_params *prm,
                    double *xo, double *po, double *co, double *chi2o, int32_t *ndfo, int32_t *sto,
                    double *margin)
{
    double xs[512], ys[512], zs[512], C[25];
    if (margin) *margin = -INFINITY;
    *ndfo = 2 * n - 5;
    if (n < 3 || n > 512) {
        *chi2o = 0.0;
        *xo = 0.0;
        for (int i = 0; i < 5; ++i) po[i] = 0.0;
        for (int i = 0; i < 15; ++i) co[i] = 0.0;
        *sto = 1;
        return;
    }
    for (int k = 0; k < n; ++k) {
        int32_t r = row0 + k;
        xs[k] = row_x[r];
        ys[k] = y[hit[k]];
        zs[k] = z[hit[k]];
        if (map) {
            ys[k] -= map[((size_t)sec * n_rows + r) * 2 + 0];
            zs[k] -= map[((size_t)sec * n_rows + r) * 2 + 1];
        }
    }
    *sto = fit_points_m(n, xs, ys, zs, prm, xo, po, C, chi2o, margin);
    pack_cov(C, co);
}

void oracle_fit(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                const int32_t *sector, const int32_t *first_row,
                const double *y, const double *z, const double *row_x, int32_t n_rows,
                const double *map, const oracle_fit_params *prm,
                double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                double *margin)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int32_t i = 0; i < n_tracks; ++i) {
        fit_one(offsets[i + 1] - offsets[i], hits + offsets[i], sector[i], first_row[i],
                y, z, row_x, n_rows, map, prm, &x_out[i], &par[(size_t)i * 5],
                &cov[(size_t)i * 15], &chi2[i], &ndf[i], &status[i], margin ? &margin[i] : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Track following.  The paper does not describe it; this is a textbook      */
/* prolongation with cluster pickup, per seed:                               */
/*  0  fit the seed as above (state at its innermost hit), each hit at the   */
/*     row of its (frame, sector) holding it, so seeds may skip rows; a seed */
/*     with a hit outside that (frame, sector) or rows not rising strictly  */
/*     is refused (status 1)                                                 */
/*  A  inwards, row by row below the innermost hit: predict to the row; stop */
/*     if the step fails or |y| exceeds the row half-width x tan 10 deg (the */
/*     track leaves the sector); among all clusters of that (frame, sector,  */
/*     row) take the one of smallest predicted-residual chi2 (ties: smaller  */
/*     id); if chi2 <= gate, update with it, else count a miss and stop      */
/*     after more than max_miss consecutive misses                           */
/*  B  outwards: restart at the innermost hit (its measured y, z, the other  */
/*     parameters from A, the start covariance of the fit), update with      */
/*     every hit above it up to the outermost, then prolong outwards above   */
/*     the outermost hit as in A                                             */
/*  C  refit all hits inwards exactly as the seed fit (three-point start at */
/*     the outermost hit, middle hit (n-1)/2 in ascending row order)         */
/* Then duplicates: each cluster belongs to the track with the smallest key  */
/* (n_rows - n_hits, track index) among the successfully refitted tracks     */
/* that hold it; a track owning fewer than half of its hits is marked 4.     */
/* margin[t] is the smallest relative distance of any floating-point         */
/* decision of A and B from its threshold (gate, tie, half-width, max_sin):  */
/* a computation with different rounding may decide differently only where   */
/* it is tiny.                                                               */
/* ------------------------------------------------------------------------ */
static double dmin(double a, double b) { return a < b ? a : b; }

/* One row of prolongation: predict p, C to plane x_r; returns 1 to go on,
 * 0 to stop.  *pick = chosen cluster or -1. */
static int follow_row(double *p, double *C, double *xcur, double xr, int32_t c0, int32_t c1,
                      const double *y, const double *z, const oracle_fit_params *prm,
                      double gate, double tan10, int32_t *pick, double *margin)
{
    double vy = prm->sigma_y * prm->sigma_y, vz = prm->sigma_z * prm->sigma_z;
    *pick = -1;
    if (predict(p, C, xr - *xcur, prm)) return 0;
    *xcur = xr;
    *margin = dmin(*margin, fabs(fabs(p[2]) - prm->max_sin));
    double hw = xr * tan10;
    *margin = dmin(*margin, fabs(fabs(p[0]) - hw) / hw);
    if (!(fabs(p[0]) <= hw)) return 0;
    double b1 = INFINITY, b2 = INFINITY;
    int32_t best = -1;
    for (int32_t c = c0; c < c1; ++c) {
        double chi = resid_chi2(p, C, y[c], z[c], vy, vz);
        if (!isfinite(chi)) continue;
        *margin = dmin(*margin, fabs(chi - gate) / (gate + 1.0));
        if (chi < b1) { b2 = b1; b1 = chi; best = c; }
        else if (chi < b2) b2 = chi;
    }
    if (best >= 0 && b1 <= gate) {
        if (b2 <= gate) *margin = dmin(*margin, (b2 - b1) / (b1 + 1.0));
        double chi2 = 0.0;
        if (update(p, C, y[best], z[best], vy, vz, &chi2)) return 0;
        *pick = best;
    }
    return 1;
}

static int32_t row_of(const int32_t *row_offsets, int32_t base, int32_t n_rows, int32_t id);

static void follow_one(int32_t i, int32_t n, const int32_t *hit, int32_t frame, int32_t sec,
                       int32_t row0, const int32_t *row_offsets, int32_t n_frames, int32_t n_sectors,
                       int32_t n_rows,
                       const double *y, const double *z, const double *row_x,
                       const oracle_fit_params *prm, const oracle_follow_params *fp,
                       int32_t *rows, double *xo, double *po, double *co, double *chi2o,
                       int32_t *ndfo, int32_t *sto, double *margin)
{
    const double tan10 = tan(3.14159265358979323846 / 18.0);   /* sector half-opening 10 deg */
    double xs[512], ys[512], zs[512], p[5], C[25];
    (void)i;
    *margin = INFINITY;
    *ndfo = 2 * n - 5;
    for (int32_t r = 0; r < n_rows; ++r) rows[r] = -1;
    /* 0: the seed fit, each hit at the row of the (frame, sector) holding it
     * (seeds from links across a missing row skip rows); a seed with a hit
     * outside its (frame, sector) or rows not rising strictly is refused */
    int refused = n < 3 || n > 512 || sec < 0 || sec >= n_sectors || frame < 0 || frame >= n_frames;
    int32_t prev = -1, base = (frame * n_sectors + sec) * n_rows;
    for (int32_t k = 0; k < n && !refused; ++k) {
        int32_t r = row_of(row_offsets, base, n_rows, hit[k]);
        if (r < 0 || r <= prev) { refused = 1; break; }
        prev = r;
        rows[r] = hit[k];
        xs[k] = row_x[r];
        ys[k] = y[hit[k]];
        zs[k] = z[hit[k]];
    }
    (void)row0;
    if (refused) {
        for (int32_t r = 0; r < n_rows; ++r) rows[r] = -1;
        *xo = 0.0;
        *chi2o = 0.0;
        for (int q = 0; q < 5; ++q) po[q] = 0.0;
        for (int q = 0; q < 15; ++q) co[q] = 0.0;
        *sto = 1;
        return;
    }
    int32_t lo = row_of(row_offsets, base, n_rows, hit[0]), hi = prev;
    *sto = fit_points(n, xs, ys, zs, prm, xo, p, C, chi2o);
    if (*sto) {
        for (int q = 0; q < 5; ++q) po[q] = p[q];
        pack_cov(C, co);
        return;
    }
    const int32_t *seg_off = row_offsets + ((size_t)frame * n_sectors + sec) * n_rows;
    /* A: inwards */
    double plo[5];
    for (int q = 0; q < 5; ++q) plo[q] = p[q];
    double xcur = row_x[lo];
    int32_t miss = 0;
    for (int32_t r = lo - 1; r >= 0; --r) {
        int32_t pick;
        if (!follow_row(p, C, &xcur, row_x[r], seg_off[r], seg_off[r + 1], y, z, prm, fp->gate,
                        tan10, &pick, margin))
            break;
        if (pick >= 0) {
            rows[r] = pick;
            lo = r;
            miss = 0;
            for (int q = 0; q < 5; ++q) plo[q] = p[q];
        } else if (++miss > fp->max_miss) {
            break;
        }
    }
    /* B: outwards from the innermost hit */
    for (int q = 0; q < 5; ++q) p[q] = plo[q];
    p[0] = y[rows[lo]];
    p[1] = z[rows[lo]];
    for (int q = 0; q < 25; ++q) C[q] = 0.0;
    C[0] = prm->sigma_y * prm->sigma_y;
    C[6] = prm->sigma_z * prm->sigma_z;
    C[12] = prm->var_sin0;
    C[18] = prm->var_tgl0;
    C[24] = prm->var_qpt0;
    xcur = row_x[lo];
    int ok = 1;
    {
        double vy = prm->sigma_y * prm->sigma_y, vz = prm->sigma_z * prm->sigma_z, chi2 = 0.0;
        for (int32_t r = lo + 1; r <= hi && ok; ++r) {
            if (rows[r] < 0) continue;
            if (predict(p, C, row_x[r] - xcur, prm)) { ok = 0; break; }
            xcur = row_x[r];
            *margin = dmin(*margin, fabs(fabs(p[2]) - prm->max_sin));
            if (update(p, C, y[rows[r]], z[rows[r]], vy, vz, &chi2)) ok = 0;
        }
    }
    if (ok) {
        miss = 0;
        for (int32_t r = hi + 1; r < n_rows; ++r) {
            int32_t pick;
            if (!follow_row(p, C, &xcur, row_x[r], seg_off[r], seg_off[r + 1], y, z, prm, fp->gate,
                            tan10, &pick, margin))
                break;
            if (pick >= 0) {
                rows[r] = pick;
                hi = r;
                miss = 0;
            } else if (++miss > fp->max_miss) {
                break;
            }
        }
    }
    /* C: refit of all hits */
    int32_t m = 0;
    for (int32_t r = lo; r <= hi; ++r) {
        if (rows[r] < 0) continue;
        xs[m] = row_x[r];
        ys[m] = y[rows[r]];
        zs[m] = z[rows[r]];
        ++m;
    }
    *sto = fit_points(m, xs, ys, zs, prm, xo, p, C, chi2o);
    for (int q = 0; q < 5; ++q) po[q] = p[q];
    pack_cov(C, co);
    *ndfo = 2 * m - 5;
}

void oracle_follow(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                   const int32_t *frame, const int32_t *sector, const int32_t *first_row,
                   const int32_t *row_offsets, int32_t n_frames, int32_t n_sectors, int32_t n_rows,
                   const double *y, const double *z, const double *row_x,
                   const oracle_fit_params *prm, const oracle_follow_params *fp,
                   int32_t *rows, double *x_out, double *par, double *cov, double *chi2,
                   int32_t *ndf, int32_t *status, double *margin)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n_tracks; ++i) {
        follow_one(i, offsets[i + 1] - offsets[i], hits + offsets[i], frame[i], sector[i],
                   first_row[i], row_offsets, n_frames, n_sectors, n_rows, y, z, row_x, prm, fp,
                   rows + (size_t)i * n_rows, &x_out[i], &par[(size_t)i * 5],
                   &cov[(size_t)i * 15], &chi2[i], &ndf[i], &status[i], &margin[i]);
    }
    /* duplicates */
    int32_t N = 0;
    for (int32_t i = 0; i < n_tracks; ++i)
        for (int32_t r = 0; r < n_rows; ++r) {
            int32_t c = rows[(size_t)i * n_rows + r];
            if (c + 1 > N) N = c + 1;
        }
    uint64_t *owner = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(N > 0 ? N : 1));
    for (int32_t c = 0; c < N; ++c) owner[c] = UINT64_MAX;
    for (int32_t i = 0; i < n_tracks; ++i) {
        if (status[i]) continue;
        uint64_t key = ((uint64_t)(uint32_t)(n_rows - (ndf[i] + 5) / 2) << 32) | (uint32_t)i;
        for (int32_t r = 0; r < n_rows; ++r) {
            int32_t c = rows[(size_t)i * n_rows + r];
            if (c >= 0 && key < owner[c]) owner[c] = key;
        }
    }
    for (int32_t i = 0; i < n_tracks; ++i) {
        if (status[i]) continue;
        int32_t nh = (ndf[i] + 5) / 2;
        uint64_t key = ((uint64_t)(uint32_t)(n_rows - nh) << 32) | (uint32_t)i;
        int32_t owned = 0;
        for (int32_t r = 0; r < n_rows; ++r) {
            int32_t c = rows[(size_t)i * n_rows + r];
            if (c >= 0 && owner[c] == key) ++owned;
        }
        if (2 * owned < nh) status[i] = 4;
    }
    free(owner);
}

/* ------------------------------------------------------------------------ */
/* Fit with material: the fit above plus multiple scattering in the gas and  */
/* rejection of outlying hits.  Before each inward step from plane a to      */
/* plane b (state at a, after its update), the scattering of the segment     */
/* between them enters the covariance: path ds = |dx| sqrt(1+t^2) /          */
/* sqrt(1-s^2), momentum p = sqrt(1+t^2)/|w|, beta = p / sqrt(p^2 + m^2),     */
/* theta0 = 0.0136/(beta p) sqrt(ds/X0) (1 + 0.038 ln(ds/X0)) (Highland), and */
/* with the two projected angles independent (phi changes by theta/cos       */
/* lambda, lambda by theta):                                                 */
/*   C_ss += th2 (1-s^2)(1+t^2), C_tt += th2 (1+t^2)^2,                     */
/*   C_tw += th2 t w (1+t^2),    C_ww += th2 t^2 w^2     (th2 = theta0^2)    */
/* (no noise for X0 infinite or w = 0).  Then, with rho > 0, the energy     */
/* loss of the segment (add_energy_loss; a particle that would stop ends    */
/* the fit with status 2), then the helix step.  After it, a hit whose       */
/* predicted-residual chi2 exceeds chi2_cut is not used (flagged; the state  */
/* goes on from the prediction).  chi2 sums the used hits, ndf = 2 used - 5  */
/* with the outermost (start) hit counted as used.  margin = smallest        */
/* |chi2 - cut| / (cut + 1) over the hits' decisions.                        */
/* ------------------------------------------------------------------------ */
static void add_scattering(const double *p, double dx, const oracle_material *m, double *C)
{
    double s = p[2], t = p[3], w = p[4];
    if (!(m->x0 < INFINITY) || w == 0.0) return;
    double t2 = 1.0 + t * t;
    double ds = fabs(dx) * sqrt(t2) / sqrt(1.0 - s * s);
    double pm = sqrt(t2) / fabs(w);
    double beta = pm / sqrt(pm * pm + m->mass * m->mass);
    double xr = ds / m->x0;
    double th = 0.0136 / (beta * pm) * sqrt(xr) * (1.0 + 0.038 * log(xr));
    double th2 = th * th;
    C[2 * 5 + 2] += th2 * (1.0 - s * s) * t2;
    C[3 * 5 + 3] += th2 * t2 * t2;
    C[3 * 5 + 4] += th2 * t * w * t2;
    C[4 * 5 + 3] += th2 * t * w * t2;
    C[4 * 5 + 4] += th2 * t * t * w * w;
}

/* Energy loss in the gas (material with rho > 0).  A segment of path ds
 * (as for the scattering) starting from state p, with momentum
 * P = sqrt(1+t^2)/|w|, energy E = sqrt(P^2 + m^2), beta = P/E and
 * gamma = E/m, loses on average ds rho <dE/dx> (Bethe, unit charge, no
 * density-effect term):
 *   <dE/dx> = K Z/A / beta^2 (ln(2 m_e beta^2 gamma^2 W / I^2) / 2 - beta^2),
 *   W = 2 m_e beta^2 gamma^2 / (1 + 2 gamma m_e/m + (m_e/m)^2)  (largest transfer),
 * K = 0.307075 MeV cm^2/mol, m_e = 0.51099895 MeV, I the mean excitation
 * energy; and the loss fluctuates with variance (Bohr, relativistic)
 *   var(E) = K Z/A rho ds m_e (1 - beta^2/2) / (1 - beta^2).
 * The particle moves outwards, so a step inwards gives back the mean loss:
 * E' = E + dE (dir = +1; the smoother's outward reference takes it away,
 * dir = -1), P' = sqrt(E'^2 - m^2), w' = w P / P' (t and s unchanged).  For
 * the covariance the loss is held fixed: w' depends on w and t through P,
 *   dw'/dw = (P/P')^3 E'/E,  dw'/dt = w' t/(1+t^2) (1 - E' P^2 / (E P'^2)),
 * and the straggling is noise on w at the start, var(E) (w E / P^2)^2.
 * A segment whose mean loss would change the momentum by more than 1 % is
 * taken without energy loss: the state's momentum is then far from any
 * track's that crosses the gas (or the particle is about to stop), and the
 * map, which contracts the q/pT variance strongly at low momentum, would
 * lock the fit onto it.
 * Returns 1 if the energy reaches the mass (the particle stops), else 0;
 * without energy loss (rho = 0, or w = 0) w' = w, J the identity, no noise. */
static double bethe(double P, double m, double zoa, double I)
{
    const double K = 0.307075e-3, me = 0.51099895e-3;     /* GeV cm^2/mol, GeV */
    double E = sqrt(P * P + m * m), b2 = P * P / (E * E), g = E / m, bg2 = P * P / (m * m);
    double W = 2.0 * me * bg2 / (1.0 + 2.0 * g * me / m + (me / m) * (me / m));
    return K * zoa / b2 * (0.5 * log(2.0 * me * bg2 * W / (I * I)) - b2);
}

double oracle_bethe(double beta_gamma, double mass, double z_over_a, double mean_exc)
{
    return bethe(beta_gamma * mass, mass, z_over_a, mean_exc);
}

static int eloss_map(const double *p, double dx, const oracle_material *m, double dir, double *wo,
                     double *J43, double *J44, double *varw)
{
    double s = p[2], t = p[3], w = p[4];
    *wo = w;
    *J43 = 0.0;
    *J44 = 1.0;
    *varw = 0.0;
    if (!(m->rho > 0.0) || w == 0.0) return 0;
    const double K = 0.307075e-3, me = 0.51099895e-3;
    double t2 = 1.0 + t * t;
    double ds = fabs(dx) * sqrt(t2) / sqrt(1.0 - s * s);
    double P = sqrt(t2) / fabs(w), E = sqrt(P * P + m->mass * m->mass), b2 = P * P / (E * E);
    double dE = ds * m->rho * bethe(P, m->mass, m->z_over_a, m->mean_exc);
    double varE = K * m->z_over_a * m->rho * ds * me * (1.0 - 0.5 * b2) / (1.0 - b2);
    double E1 = E + dir * dE;
    if (!(E1 > m->mass)) return 1;
    double P1 = sqrt(E1 * E1 - m->mass * m->mass);
    if (fabs(P1 - P) > 0.01 * P) return 0;
    *wo = w * P / P1;
    *J44 = (P / P1) * (P / P1) * (P / P1) * E1 / E;
    *J43 = *wo * t / t2 * (1.0 - E1 * P * P / (E * P1 * P1));
    double dw = w * E / (P * P);
    *varw = varE * dw * dw;
    return 0;
}

int32_t oracle_eloss(const double *p, double dx, const oracle_material *m, double dir, double *out)
{
    return eloss_map(p, dx, m, dir, &out[0], &out[1], &out[2], &out[3]);
}

/* The energy loss of the segment dx in a fit step inwards: straggling
 * noise added to C, then p, C moved by the map (C <- J C J^T).  Returns 1
 * if the particle would stop. */
static int add_energy_loss(double *p, double *C, double dx, const oracle_material *m)
{
    double w1, j43, j44, vw;
    if (eloss_map(p, dx, m, 1.0, &w1, &j43, &j44, &vw)) return 1;
    double J[25] = {0}, Jt[25], T[25];
    for (int i = 0; i < 5; ++i) J[i * 5 + i] = 1.0;
    J[4 * 5 + 3] = j43;
    J[4 * 5 + 4] = j44;
    C[24] += vw;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Jt[i * 5 + j] = J[j * 5 + i];
    mat5_mul(J, C, T);
    mat5_mul(T, Jt, C);
    p[4] = w1;
    return 0;
}

/* Fit with material of n points at planes xs (ascending), point k with the
 * measurement variances vys[k], vzs[k] (the outermost point's are also the
 * start covariance of y and z). */
static void fit_material_points(int32_t n, const double *xs, const double *ys, const double *zs,
                                const double *vys, const double *vzs, const oracle_fit_params *prm,
                                const oracle_material *mat, double *xo, double *po, double *co,
                                double *chi2o, int32_t *ndfo, int32_t *sto, uint8_t *rej, double *margin)
{
    double C[25], p[5];
    int32_t st = start_points(n, xs, ys, zs, prm, p, C);
    C[0] = vys[n - 1];
    C[6] = vzs[n - 1];
    double chi2 = 0.0, xcur = xs[n - 1];
    int32_t used = 1;
    for (int k = n - 2; k >= 0 && !st; --k) {
        double dx = xs[k] - xs[k + 1];
        add_scattering(p, dx, mat, C);
        if (add_energy_loss(p, C, dx, mat)) { st = 2; break; }
        if (predict(p, C, dx, prm)) { st = 2; break; }
        xcur = xs[k];
        double chi = resid_chi2(p, C, ys[k], zs[k], vys[k], vzs[k]);
        if (isfinite(chi)) {
            double mg = fabs(chi - mat->chi2_cut) / (mat->chi2_cut + 1.0);
            if (mg < *margin) *margin = mg;
        }
        if (chi > mat->chi2_cut) {
            rej[k] = 1;
        } else {
            if (update(p, C, ys[k], zs[k], vys[k], vzs[k], &chi2)) { st = 3; break; }
            ++used;
        }
    }
    *xo = xcur;
    for (int i = 0; i < 5; ++i) po[i] = p[i];
    pack_cov(C, co);
    *chi2o = chi2;
    *ndfo = 2 * used - 5;
    *sto = st;
}

/* Outputs of a refused seed (status 1). */
static void refuse(int32_t n, double *xo, double *po, double *co, double *chi2o, int32_t *ndfo,
                   int32_t *sto, uint8_t *rej, double *margin)
{
    *margin = INFINITY;
    for (int k = 0; k < n && k < 512; ++k) rej[k] = 0;
    *ndfo = 2 * n - 5;
    *chi2o = 0.0;
    *xo = 0.0;
    for (int i = 0; i < 5; ++i) po[i] = 0.0;
    for (int i = 0; i < 15; ++i) co[i] = 0.0;
    *sto = 1;
}

static void fit_one_material(int32_t n, const int32_t *hit, int32_t row0, const double *y, const double *z,
                             const double *row_x, const oracle_fit_params *prm, const oracle_material *mat,
                             double *xo, double *po, double *co, double *chi2o, int32_t *ndfo, int32_t *sto,
                             uint8_t *rej, double *margin)
{
    double xs[512], ys[512], zs[512], vys[512], vzs[512];
    refuse(n, xo, po, co, chi2o, ndfo, sto, rej, margin);
    if (n < 3 || n > 512) return;
    double vy = prm->sigma_y * prm->sigma_y, vz = prm->sigma_z * prm->sigma_z;
    for (int k = 0; k < n; ++k) {
        xs[k] = row_x[row0 + k];
        ys[k] = y[hit[k]];
        zs[k] = z[hit[k]];
        vys[k] = vy;
        vzs[k] = vz;
    }
    fit_material_points(n, xs, ys, zs, vys, vzs, prm, mat, xo, po, co, chi2o, ndfo, sto, rej, margin);
}

void oracle_fit_material(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                         const int32_t *first_row, const double *y, const double *z, const double *row_x,
                         const oracle_fit_params *prm, const oracle_material *mat,
                         double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                         uint8_t *rejected, double *margin)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int32_t i = 0; i < n_tracks; ++i) {
        fit_one_material(offsets[i + 1] - offsets[i], hits + offsets[i], first_row[i], y, z, row_x, prm, mat,
                         &x_out[i], &par[(size_t)i * 5], &cov[(size_t)i * 15], &chi2[i], &ndf[i], &status[i],
                         rejected + offsets[i], &margin[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Fit of seeds whose hits may skip pad rows, with per-cluster errors.        */
/* The row of a hit is the pad row of the seed's (frame, sector) whose id     */
/* range holds it; a seed with a hit outside that (frame, sector), or whose   */
/* rows do not rise strictly with the hit index, is refused (status 1).  Hit  */
/* h is measured with variances err[h][0]^2, err[h][1]^2 (err null: sigma_y^2 */
/* and sigma_z^2 for every hit), which also enter the start covariance at     */
/* the outermost hit.  Otherwise this is the fit with material above, and     */
/* with an infinite radiation length and no cut the plain fit.  When asked,  */
/* the smoother about the fit's trajectory (smooth_reference) then gives the */
/* state at every hit's plane from all hits; a failing smoother step sets    */
/* status 2 or 3 and zero smoothed states.                                   */
/* ------------------------------------------------------------------------ */

/* Pad row of cluster id among the rows [base, base + n_rows) of one
 * (frame, sector), or -1 if the id lies in none of them. */
static int32_t row_of(const int32_t *row_offsets, int32_t base, int32_t n_rows, int32_t id)
{
    if (id < row_offsets[base] || id >= row_offsets[base + n_rows]) return -1;
    int32_t lo = 0, hi = n_rows - 1;          /* off[base+lo] <= id < off[base+hi+1] */
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (row_offsets[base + mid] <= id) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

/* Inverse of a 5x5 matrix by Gauss-Jordan elimination with partial
 * pivoting; returns 0, or 1 if a pivot vanishes. */
static int inv5(const double *A, double *X)
{
    double M[5][10];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 10; ++j) M[i][j] = j < 5 ? A[i * 5 + j] : (j - 5 == i ? 1.0 : 0.0);
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int i = c + 1; i < 5; ++i)
            if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
        if (!(fabs(M[piv][c]) > 0.0)) return 1;
        if (piv != c)
            for (int j = 0; j < 10; ++j) { double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t; }
        double d = M[c][c];
        for (int j = 0; j < 10; ++j) M[c][j] /= d;
        for (int i = 0; i < 5; ++i) {
            if (i == c) continue;
            double f = M[i][c];
            for (int j = 0; j < 10; ++j) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) X[i * 5 + j] = M[i][j + 5];
    return 0;
}

/* Smoother about a reference trajectory.  The reference starts at the
 * outermost plane from the fit's final state carried there -- by one exact
 * helix step, or, with energy loss, plane by plane with the helix step and
 * the loss of each segment taken away -- and runs inwards by the fit's own
 * step (energy loss, then helix step): r_{k-1} = f(r_k) (a step or a loss
 * that fails ends the smoothing with status 2).  About it the problem is
 * linear in the deviation d = state - r: the step from plane k to plane k-1
 * maps d by its Jacobian F_k (helix step times energy loss, taken on the
 * reference), the scattering and the straggling of that segment add Q_k
 * (from r_k) before the step, and a hit measures (y, z) of r + d.  A Kalman filter of d runs inwards from plane n-1 (d = 0,
 * variances (100 sigma)^2 on y and z and the start variances on the other
 * three), taking the hits the fit used (none it rejected); then the
 * Rauch-Tung-Striebel pass outwards:
 *   G = C_k F_k^T P^-1,  P = F_k (C_k + Q_k) F_k^T,
 *   d_s(k) = d_k + G (d_s(k-1) - F_k d_k),
 *   C_s(k) = C_k + G (C_s(k-1) - P) G^T,
 * starting from the filtered d at plane 0.  The smoothed state is r_k +
 * d_s(k), written to sp[n][5], sc[n][15] (packed).  Returns 0, 2 or 3. */
static int32_t smooth_reference(int32_t n, const double *xs, const double *ys, const double *zs,
                                const double *vys, const double *vzs, const uint8_t *rej, const double *pfin,
                                const oracle_fit_params *prm, const oracle_material *mat,
                                double *sp, double *sc)
{
    /* per plane: reference state (5), Jacobian of the step inwards from it
     * (25), scattering covariance of that segment (25), filtered d (5) and
     * covariance (25) */
    double *w = (double *)malloc(sizeof(double) * (size_t)n * 85);
    double *R = w, *FJ = w + (size_t)n * 5, *QS = w + (size_t)n * 30, *D = w + (size_t)n * 55,
           *CD = w + (size_t)n * 60;
    int32_t st = 0;
    double *Rn = R + (size_t)(n - 1) * 5, F[25];
    if (mat->rho > 0.0) {                      /* the outermost reference state */
        double a[5], j43, j44, vw;
        memcpy(a, pfin, sizeof a);
        for (int k = 1; k < n && !st; ++k) {
            double dx = xs[k] - xs[k - 1];
            if (oracle_propagate(a, dx, prm->bz, prm->max_sin, Rn, F) ||
                eloss_map(Rn, dx, mat, -1.0, &Rn[4], &j43, &j44, &vw)) st = 2;
            memcpy(a, Rn, sizeof a);
        }
    } else if (oracle_propagate(pfin, xs[n - 1] - xs[0], prm->bz, prm->max_sin, Rn, F)) {
        st = 2;
    }
    for (int k = n - 1; k >= 1 && !st; --k) {  /* steps inwards along it */
        double dx = xs[k - 1] - xs[k], w1, j43, j44, vw, re[5], J[25] = {0};
        const double *r = R + (size_t)k * 5;
        double *Q = QS + (size_t)k * 25;
        for (int i = 0; i < 25; ++i) Q[i] = 0.0;
        add_scattering(r, dx, mat, Q);
        if (eloss_map(r, dx, mat, 1.0, &w1, &j43, &j44, &vw)) { st = 2; break; }
        Q[24] += vw;
        memcpy(re, r, sizeof re);
        re[4] = w1;
        for (int i = 0; i < 5; ++i) J[i * 5 + i] = 1.0;
        J[4 * 5 + 3] = j43;
        J[4 * 5 + 4] = j44;
        if (oracle_propagate(re, dx, prm->bz, prm->max_sin, R + (size_t)(k - 1) * 5, F)) { st = 2; break; }
        mat5_mul(F, J, FJ + (size_t)k * 25);
    }
    /* inward filter of the deviation */
    double d[5] = {0, 0, 0, 0, 0}, C[25], chi2 = 0.0;
    for (int i = 0; i < 25; ++i) C[i] = 0.0;
    C[0] = 1e4 * vys[n - 1];
    C[6] = 1e4 * vzs[n - 1];
    C[12] = prm->var_sin0;
    C[18] = prm->var_tgl0;
    C[24] = prm->var_qpt0;
    for (int k = n - 1; k >= 0 && !st; --k) {
        if (k < n - 1) {
            const double *F = FJ + (size_t)(k + 1) * 25, *Q = QS + (size_t)(k + 1) * 25;
            double Ft[25], T[25], nd[5];
            for (int i = 0; i < 25; ++i) C[i] += Q[i];
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j < 5; ++j) Ft[i * 5 + j] = F[j * 5 + i];
            mat5_mul(F, C, T);
            mat5_mul(T, Ft, C);
            for (int i = 0; i < 5; ++i) {
                double acc = 0.0;
                for (int j = 0; j < 5; ++j) acc += F[i * 5 + j] * d[j];
                nd[i] = acc;
            }
            memcpy(d, nd, sizeof d);
        }
        if (!rej[k]) {
            /* the hit measures r + d: update d with the residual about r */
            const double *r = R + (size_t)k * 5;
            double md[5];
            memcpy(md, d, sizeof md);
            if (update(md, C, ys[k] - r[0], zs[k] - r[1], vys[k], vzs[k], &chi2)) st = 3;
            memcpy(d, md, sizeof d);
        }
        memcpy(D + (size_t)k * 5, d, sizeof d);
        memcpy(CD + (size_t)k * 25, C, sizeof C);
    }
    if (!st) {
        /* outwards: Rauch-Tung-Striebel */
        double ds[5], Cs[25];
        memcpy(ds, D, sizeof ds);
        memcpy(Cs, CD, sizeof Cs);
        for (int i = 0; i < 5; ++i) sp[i] = R[i] + ds[i];
        pack_cov(Cs, sc);
        for (int k = 1; k < n && !st; ++k) {
            const double *F = FJ + (size_t)k * 25, *Q = QS + (size_t)k * 25;
            const double *dk = D + (size_t)k * 5, *Ck = CD + (size_t)k * 25;
            double Cq[25], Ft[25], T[25], P[25], Pi[25], G[25], Gt[25], E[25], GE[25], pd[5];
            for (int i = 0; i < 25; ++i) Cq[i] = Ck[i] + Q[i];
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j < 5; ++j) Ft[i * 5 + j] = F[j * 5 + i];
            mat5_mul(F, Cq, T);
            mat5_mul(T, Ft, P);
            if (inv5(P, Pi)) { st = 3; break; }
            mat5_mul(Ck, Ft, T);
            mat5_mul(T, Pi, G);
            for (int i = 0; i < 5; ++i) {
                double acc = 0.0;
                for (int j = 0; j < 5; ++j) acc += F[i * 5 + j] * dk[j];
                pd[i] = acc;
            }
            double nds[5];
            for (int i = 0; i < 5; ++i) {
                double acc = dk[i];
                for (int j = 0; j < 5; ++j) acc += G[i * 5 + j] * (ds[j] - pd[j]);
                nds[i] = acc;
            }
            for (int i = 0; i < 25; ++i) E[i] = Cs[i] - P[i];
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j < 5; ++j) Gt[i * 5 + j] = G[j * 5 + i];
            mat5_mul(G, E, T);
            mat5_mul(T, Gt, GE);
            for (int i = 0; i < 25; ++i) Cs[i] = Ck[i] + GE[i];
            memcpy(ds, nds, sizeof ds);
            for (int i = 0; i < 5; ++i) sp[(size_t)k * 5 + i] = R[(size_t)k * 5 + i] + ds[i];
            pack_cov(Cs, sc + (size_t)k * 15);
        }
    }
    free(w);
    return st;
}

static void fit_one_rows(int32_t n, const int32_t *hit, int32_t frame, int32_t sec,
                         const int32_t *row_offsets, int32_t n_frames, int32_t n_sectors, int32_t n_rows,
                         const double *y, const double *z, const double *row_x, const float *err,
                         const oracle_fit_params *prm, const oracle_material *mat,
                         double *xo, double *po, double *co, double *chi2o, int32_t *ndfo, int32_t *sto,
                         uint8_t *rej, double *margin, double *sp, double *sc)
{
    double xs[512], ys[512], zs[512], vys[512], vzs[512];
    refuse(n, xo, po, co, chi2o, ndfo, sto, rej, margin);
    if (sp)
        for (int k = 0; k < n && k < 512; ++k) {
            for (int i = 0; i < 5; ++i) sp[(size_t)k * 5 + i] = 0.0;
            for (int i = 0; i < 15; ++i) sc[(size_t)k * 15 + i] = 0.0;
        }
    if (n < 3 || n > 512 || frame < 0 || frame >= n_frames || sec < 0 || sec >= n_sectors) return;
    int32_t base = (frame * n_sectors + sec) * n_rows;
    int32_t prev = -1;
    for (int k = 0; k < n; ++k) {
        int32_t r = row_of(row_offsets, base, n_rows, hit[k]);
        if (r < 0 || r <= prev) return;
        prev = r;
        xs[k] = row_x[r];
        ys[k] = y[hit[k]];
        zs[k] = z[hit[k]];
        if (err) {
            double ey = (double)err[(size_t)hit[k] * 2], ez = (double)err[(size_t)hit[k] * 2 + 1];
            vys[k] = ey * ey;
            vzs[k] = ez * ez;
        } else {
            vys[k] = prm->sigma_y * prm->sigma_y;
            vzs[k] = prm->sigma_z * prm->sigma_z;
        }
    }
    if (!sp) {
        fit_material_points(n, xs, ys, zs, vys, vzs, prm, mat, xo, po, co, chi2o, ndfo, sto, rej, margin);
        return;
    }
    fit_material_points(n, xs, ys, zs, vys, vzs, prm, mat, xo, po, co, chi2o, ndfo, sto, rej, margin);
    if (*sto == 0) {
        int32_t s2 = smooth_reference(n, xs, ys, zs, vys, vzs, rej, po, prm, mat, sp, sc);
        if (s2) {
            *sto = s2;
            for (int k = 0; k < n; ++k) {
                for (int i = 0; i < 5; ++i) sp[(size_t)k * 5 + i] = 0.0;
                for (int i = 0; i < 15; ++i) sc[(size_t)k * 15 + i] = 0.0;
            }
        }
    }
}

void oracle_fit_rows(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                     const int32_t *frame, const int32_t *sector, const int32_t *row_offsets,
                     int32_t n_frames, int32_t n_sectors, int32_t n_rows,
                     const double *y, const double *z, const double *row_x, const float *err,
                     const oracle_fit_params *prm, const oracle_material *mat,
                     double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                     uint8_t *rejected, double *margin, double *hit_par, double *hit_cov)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int32_t i = 0; i < n_tracks; ++i) {
        fit_one_rows(offsets[i + 1] - offsets[i], hits + offsets[i], frame[i], sector[i], row_offsets,
                     n_frames, n_sectors, n_rows, y, z, row_x, err, prm, mat, &x_out[i], &par[(size_t)i * 5],
                     &cov[(size_t)i * 15], &chi2[i], &ndf[i], &status[i], rejected + offsets[i], &margin[i],
                     hit_par ? hit_par + (size_t)offsets[i] * 5 : NULL,
                     hit_cov ? hit_cov + (size_t)offsets[i] * 15 : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Merging of track segments across sector edges (a step after the fit that */
/* the paper implies but gives no algorithm for).  A particle that crosses  */
/* from one sector into the next on the same side leaves a fitted segment   */
/* in each; their states, carried to a common plane, agree within their     */
/* covariances.                                                             */
/*  transfer  the state p at plane x of one sector's frame, rotated into the */
/*            frame turned by da (a point (x, y) -> (x cos da + y sin da,     */
/*            -x sin da + y cos da), phi -> phi - da with cos phi > 0 kept),  */
/*            then carried along the helix to plane xt of that frame.  Its   */
/*            Jacobian: the step's (at fixed distance) times the rotation's   */
/*            (dy'/dy = cos da, ds'/ds = cos da + (s/c) sin da), plus the     */
/*            move of the start plane with y (dx'/dy = sin da), which         */
/*            shortens the step: minus the end state's derivative along x     */
/*            (s/c, t/c, kappa, 0, 0) times sin da in the y column.           */
/*  pairs     fitted segments (status 0) A, B of one frame in neighbouring    */
/*            sectors of one side, A's innermost point at the smaller radius: */
/*            chi2 = d^T (J C_A J^T + C_B)^-1 d, d = transfer(A to B's        */
/*            innermost plane) - p_B.  (t and q/pT are unchanged by the       */
/*            transfer, so a pair whose t or q/pT difference alone exceeds    */
/*            the cut in its own variance cannot pass and is not computed.)   */
/*  links     A's best outer partner is the B of smallest chi2 <= cut (the   */
/*            smaller index on ties), B's best inner partner likewise; A and  */
/*            B are linked when each is the other's best: next[A] = B,        */
/*            prev[B] = A, chi2[A] = the pair's chi2; else -1 (chi2 0).       */
/*  refit     for a linked A, the two segments combined at B's plane: A's     */
/*            transferred state (covariance P = J C_A J^T) and B's, each      */
/*            independent of the other, fused by x = p_A' + P S^-1 (p_B -     */
/*            p_A'), C = P S^-1 C_B (= P - P S^-1 P), S = P + C_B -- the      */
/*            joint fit of both segments' hits for the linearised problem    */
/*            (zeros if unlinked).                                           */
/* ------------------------------------------------------------------------ */
int32_t oracle_transfer(const double *p, double x, double da, double xt, double bz, double max_sin,
                        double *pout, double *J)
{
    double y = p[0], s = p[2];
    if (!(fabs(s) < 1.0)) return 2;
    double c = sqrt(1.0 - s * s), ca = cos(da), sa = sin(da);
    double x1 = x * ca + y * sa;
    double q[5] = {-x * sa + y * ca, p[1], s * ca - c * sa, p[3], p[4]};
    if (!(c * ca + s * sa > 0.0)) return 2;
    double F[25];
    if (oracle_propagate(q, xt - x1, bz, max_sin, pout, J ? F : NULL)) return 2;
    if (J) {
        double Rm[25] = {0};
        for (int i = 0; i < 5; ++i) Rm[i * 5 + i] = 1.0;
        Rm[0] = ca;
        Rm[2 * 5 + 2] = ca + s / c * sa;
        mat5_mul(F, Rm, J);
        double s2 = pout[2], c2 = sqrt(1.0 - s2 * s2);
        double v[5] = {s2 / c2, p[3] / c2, -C_LIGHT * bz * p[4], 0.0, 0.0};
        for (int i = 0; i < 5; ++i) J[i * 5 + 0] -= v[i] * sa;
    }
    return 0;
}

#define PI_D 3.14159265358979323846

static void unpack_cov(const double *co, double *C)
{
    for (int i = 0, k = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j, ++k) C[i * 5 + j] = C[j * 5 + i] = co[k];
}

static double sector_angle(int32_t sec, int32_t n_sectors)
{
    return n_sectors == 1 ? 0.0 : (double)(sec % 18) * (PI_D / 9.0) + PI_D / 18.0;
}

/* chi2 of carrying track a onto track b (INFINITY if it cannot be formed);
 * with mp, mc non-null also the two combined at b's plane (the transferred
 * state of a, covariance P = J C_a J^T, and b's: x = p_a' + P S^-1 (p_b -
 * p_a'), C = P S^-1 C_b, which equals P - P S^-1 P but has no difference
 * of large terms, symmetrised; S = P + C_b; packed). */
static double pair_fuse(int32_t a, int32_t b, const double *x, const double *par, const double *cov,
                        const int32_t *sector, int32_t n_sectors, double bz, double max_sin, double *mp,
                        double *mc)
{
    double da = sector_angle(sector[b], n_sectors) - sector_angle(sector[a], n_sectors);
    if (da > PI_D) da -= 2.0 * PI_D;
    if (da < -PI_D) da += 2.0 * PI_D;
    double pa[5], J[25], Ca[25], Cb[25], T1[25], Jt[25], S[25], Si[25], d[5];
    unpack_cov(cov + (size_t)a * 15, Ca);
    unpack_cov(cov + (size_t)b * 15, Cb);
    if (oracle_transfer(par + (size_t)a * 5, x[a], da, x[b], bz, max_sin, pa, J)) return INFINITY;
    double P[25];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Jt[i * 5 + j] = J[j * 5 + i];
    mat5_mul(J, Ca, T1);
    mat5_mul(T1, Jt, P);
    for (int i = 0; i < 25; ++i) S[i] = P[i] + Cb[i];
    if (inv5(S, Si)) return INFINITY;
    for (int i = 0; i < 5; ++i) d[i] = pa[i] - par[(size_t)b * 5 + i];
    double chi = 0.0;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) chi += d[i] * Si[i * 5 + j] * d[j];
    if (mp && mc) {
        double K[25], C[25];
        mat5_mul(P, Si, K);                        /* K = P S^-1 */
        for (int i = 0; i < 5; ++i) {
            double acc = pa[i];
            for (int j = 0; j < 5; ++j) acc -= K[i * 5 + j] * d[j];   /* d = p_a' - p_b */
            mp[i] = acc;
        }
        /* C = P S^-1 C_b (= C_b S^-1 P), symmetrised: no difference of two
         * large terms when one segment's covariance dwarfs the other's */
        double SC[25], PSC[25], CSP[25];
        mat5_mul(Si, Cb, SC);
        mat5_mul(P, SC, PSC);
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) CSP[i * 5 + j] = PSC[j * 5 + i];
        for (int i = 0; i < 25; ++i) C[i] = 0.5 * (PSC[i] + CSP[i]);
        pack_cov(C, mc);
    }
    return chi > 0.0 ? chi : INFINITY;
}

static double pair_chi2(int32_t a, int32_t b, const double *x, const double *par, const double *cov,
                        const int32_t *sector, int32_t n_sectors, double bz, double max_sin)
{
    return pair_fuse(a, b, x, par, cov, sector, n_sectors, bz, max_sin, NULL, NULL);
}

static int neighbours_of(int32_t sa, int32_t sb, int32_t n_sectors)
{
    if (n_sectors != 36 || sa / 18 != sb / 18) return 0;
    int32_t d = ((sb % 18) - (sa % 18) + 18) % 18;
    return d == 1 || d == 17;
}

void oracle_merge(int32_t n_tracks, const double *x, const double *par, const double *cov, const int32_t *status,
                  const int32_t *frame, const int32_t *sector, int32_t n_sectors, double bz, double max_sin,
                  double cut, int32_t *next, int32_t *prev, double *chi2, double *mpar, double *mcov)
{
    int32_t *bo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_tracks ? n_tracks : 1));
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_tracks ? n_tracks : 1));
    double *co = (double *)malloc(sizeof(double) * (size_t)(n_tracks ? n_tracks : 1));
    double *ci = (double *)malloc(sizeof(double) * (size_t)(n_tracks ? n_tracks : 1));
    for (int32_t i = 0; i < n_tracks; ++i) { bo[i] = bi[i] = -1; co[i] = ci[i] = INFINITY; }
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t a = 0; a < n_tracks; ++a) {
        if (status[a]) continue;
        double ra = hypot(x[a], par[(size_t)a * 5]);
        for (int32_t b = 0; b < n_tracks; ++b) {
            if (status[b] || frame[b] != frame[a] || !neighbours_of(sector[a], sector[b], n_sectors)) continue;
            double rb = hypot(x[b], par[(size_t)b * 5]);
            /* a is the inner segment of the pair */
            const double *ca = cov + (size_t)a * 15, *cb = cov + (size_t)b * 15;
            double dt = par[(size_t)a * 5 + 3] - par[(size_t)b * 5 + 3];
            double dw = par[(size_t)a * 5 + 4] - par[(size_t)b * 5 + 4];
            if (dt * dt > cut * (ca[9] + cb[9]) || dw * dw > cut * (ca[14] + cb[14])) continue;
            if (ra < rb) {
                double chi = pair_chi2(a, b, x, par, cov, sector, n_sectors, bz, max_sin);
                if (chi <= cut && chi < co[a]) { co[a] = chi; bo[a] = b; }
            } else if (rb < ra) {
                double chi = pair_chi2(b, a, x, par, cov, sector, n_sectors, bz, max_sin);
                if (chi <= cut && chi < ci[a]) { ci[a] = chi; bi[a] = b; }
            }
        }
    }
    for (int32_t a = 0; a < n_tracks; ++a) {
        int32_t b = bo[a];
        int linked = b >= 0 && bi[b] == a;
        next[a] = linked ? b : -1;
        chi2[a] = linked ? co[a] : 0.0;
    }
    for (int32_t b = 0; b < n_tracks; ++b) {
        int32_t a = bi[b];
        prev[b] = (a >= 0 && next[a] == b) ? a : -1;
    }
    if (mpar && mcov)
        for (int32_t a = 0; a < n_tracks; ++a) {
            double *mp = mpar + (size_t)a * 5, *mc = mcov + (size_t)a * 15;
            for (int i = 0; i < 5; ++i) mp[i] = 0.0;
            for (int i = 0; i < 15; ++i) mc[i] = 0.0;
            if (next[a] >= 0)
                pair_fuse(a, next[a], x, par, cov, sector, n_sectors, bz, max_sin, mp, mc);
        }
    free(bo); free(bi); free(co); free(ci);
}

/* ------------------------------------------------------------------------ */
/* Legs of loopers.  A particle whose circle stays inside the TPC turns back */
/* inwards; the returning leg is fitted as a track running outwards, i.e.   */
/* along the same circle in the other sense: its fitted q/pT and tan lambda */
/* have the opposite signs, its circle centre is the same point.  Each       */
/* segment's circle: curvature kappa = -c Bz w, centre (x - s/kappa,         */
/* y + sqrt(1-s^2)/kappa) in its frame, turned to global coordinates by its */
/* sector angle.  m = (X_c, Y_c, kappa, t); for two legs of one particle     */
/* m_A - D m_B = 0 with D = diag(1, 1, -1, -1).  chi2 = d^T (J_A C_A J_A^T + */
/* D J_B C_B J_B^T D)^-1 d (4 degrees of freedom), J the Jacobian of m in   */
/* (y, z, s, t, w).  Candidates: fitted segments (status 0) of one frame and */
/* side, in any sectors (the legs' seeded pieces lie far apart in azimuth),  */
/* both with a circle radius                                                 */
/* below 250 cm (only a circle smaller than the TPC can return; the margin   */
/* keeps poorly measured radii).  Partners are mutual best below the cut    */
/* (smaller index on ties): leg[A] = B, leg[B] = A, leg_chi2 the pair's     */
/* chi2; else -1 and 0.                                                      */
/* ------------------------------------------------------------------------ */
#define LEG_MAX_RADIUS 250.0

/* m and its Jacobian (4x5, row-major) for one segment; returns 1 if its
 * circle is too large or the state is degenerate. */
int32_t oracle_leg_circle(const double *p, double x, double alpha, double bz, double *m, double *J)
{
    double y = p[0], s = p[2], t = p[3], w = p[4];
    double k = -C_LIGHT * bz, kap = k * w;
    if (!(fabs(s) < 1.0) || !(fabs(kap) * LEG_MAX_RADIUS > 1.0)) return 1;
    double c = sqrt(1.0 - s * s), ca = cos(alpha), sa = sin(alpha);
    double xc = x - s / kap, yc = y + c / kap;
    m[0] = xc * ca - yc * sa;
    m[1] = xc * sa + yc * ca;
    m[2] = kap;
    m[3] = t;
    if (J) {
        /* local centre: d xc = (0, 0, -1/kap, 0, s k / kap^2), d yc = (1, 0, -s/(c kap), 0, -c k / kap^2) */
        double dxc[5] = {0.0, 0.0, -1.0 / kap, 0.0, s * k / (kap * kap)};
        double dyc[5] = {1.0, 0.0, -s / (c * kap), 0.0, -c * k / (kap * kap)};
        for (int j = 0; j < 5; ++j) {
            J[0 * 5 + j] = dxc[j] * ca - dyc[j] * sa;
            J[1 * 5 + j] = dxc[j] * sa + dyc[j] * ca;
            J[2 * 5 + j] = j == 4 ? k : 0.0;
            J[3 * 5 + j] = j == 3 ? 1.0 : 0.0;
        }
    }
    return 0;
}

static int inv4(const double *A, double *X)
{
    double M[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) M[i][j] = j < 4 ? A[i * 4 + j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int i = c + 1; i < 4; ++i)
            if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
        if (!(fabs(M[piv][c]) > 0.0)) return 1;
        if (piv != c)
            for (int j = 0; j < 8; ++j) { double q = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = q; }
        double d = M[c][c];
        for (int j = 0; j < 8; ++j) M[c][j] /= d;
        for (int i = 0; i < 4; ++i) {
            if (i == c) continue;
            double f = M[i][c];
            for (int j = 0; j < 8; ++j) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) X[i * 4 + j] = M[i][j + 4];
    return 0;
}

/* J C J^T (4x4) of a segment's packed covariance. */
static void leg_cov(const double *J, const double *co, double *out)
{
    double C[25], JC[20];
    unpack_cov(co, C);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 5; ++k) acc += J[i * 5 + k] * C[k * 5 + j];
            JC[i * 5 + j] = acc;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 5; ++k) acc += JC[i * 5 + k] * J[j * 5 + k];
            out[i * 4 + j] = acc;
        }
}

static int leg_candidates(int32_t sa, int32_t sb, int32_t n_sectors)
{
    return n_sectors == 36 && sa / 18 == sb / 18;
}

void oracle_legs(int32_t n_tracks, const double *x, const double *par, const double *cov, const int32_t *status,
                 const int32_t *frame, const int32_t *sector, int32_t n_sectors, double bz, double cut,
                 int32_t *leg, double *leg_chi2)
{
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_tracks ? n_tracks : 1));
    double *bchi = (double *)malloc(sizeof(double) * (size_t)(n_tracks ? n_tracks : 1));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t a = 0; a < n_tracks; ++a) {
        best[a] = -1;
        bchi[a] = INFINITY;
        double ma[4], Ja[20], Sa[16];
        if (status[a] || oracle_leg_circle(par + (size_t)a * 5, x[a], sector_angle(sector[a], n_sectors), bz, ma, Ja))
            continue;
        leg_cov(Ja, cov + (size_t)a * 15, Sa);
        for (int32_t b = 0; b < n_tracks; ++b) {
            double mb[4], Jb[20], Sb[16], S[16], Si[16], d[4];
            if (b == a || status[b] || frame[b] != frame[a] || !leg_candidates(sector[a], sector[b], n_sectors))
                continue;
            if (oracle_leg_circle(par + (size_t)b * 5, x[b], sector_angle(sector[b], n_sectors), bz, mb, Jb)) continue;
            leg_cov(Jb, cov + (size_t)b * 15, Sb);
            /* D Sb D flips the signs of the (centre, kappa/t) cross terms */
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    double sg = ((i < 2) == (j < 2)) ? 1.0 : -1.0;
                    S[i * 4 + j] = Sa[i * 4 + j] + sg * Sb[i * 4 + j];
                }
            d[0] = ma[0] - mb[0];
            d[1] = ma[1] - mb[1];
            d[2] = ma[2] + mb[2];
            d[3] = ma[3] + mb[3];
            if (d[2] * d[2] > cut * S[10] || d[3] * d[3] > cut * S[15]) continue;
            if (inv4(S, Si)) continue;
            double chi = 0.0;
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) chi += d[i] * Si[i * 4 + j] * d[j];
            if (chi > 0.0 && chi <= cut && chi < bchi[a]) { bchi[a] = chi; best[a] = b; }
        }
    }
    for (int32_t a = 0; a < n_tracks; ++a) {
        int32_t b = best[a];
        int linked = b >= 0 && best[b] == a;
        leg[a] = linked ? b : -1;
        leg_chi2[a] = linked ? bchi[a] : 0.0;
    }
    free(best);
    free(bchi);
}

/* ------------------------------------------------------------------------ */
/* Tracks assembled from linked segments and refitted over all their hits   */
/* (a step after merging that the paper implies but does not describe).     */
/*  links     a next link i -> j counts when j = next[i] is a segment other  */
/*            than i with prev[j] = i and both fits have status 0; a leg     */
/*            link i -- j when leg[j] = i likewise.                          */
/*  track id  the connected components of the segments of status 0 under    */
/*            both kinds of link, each named by its smallest segment index  */
/*            (-1 for a segment whose own fit failed).                       */
/*  chains    a head is a segment of status 0 with no counted prev link; its */
/*            chain follows the next links outwards (at most 18 segments,    */
/*            one per sector of a side; longer: status 6).  Its hits, k =    */
/*            0..n-1, are the head's in ascending row, then the next         */
/*            segment's, and so on, each measured in its own sector's frame  */
/*            (corrected by the map of its sector and row when one is given).*/
/*  refit     the seed fit of that hit list: the exact circle through hits   */
/*            n-1, (n-1)/2 and 0, all turned into the frame of hit n-1 (a    */
/*            point (x, y) of a sector at angle a_s seen from the frame at    */
/*            angle a_t: (x cos d - y sin d, x sin d + y cos d), d = a_s -   */
/*            a_t), gives the start at hit n-1 with the start covariance;    */
/*            the filter then runs inwards, k = n-2 .. 0: within a segment   */
/*            the helix step to the plane of hit k, across a segment         */
/*            boundary the transfer above into the frame of hit k's segment  */
/*            and on to its plane (C <- J C J^T), then the update.  Written  */
/*            at the head: the state at its innermost hit in its frame, chi2,*/
/*            ndf = 2n - 5, status as the fit's; every other segment gets   */
/*            status 5 and zeros.  A chain of one segment is that segment's */
/*            seed fit.                                                      */
/*  loopers   for each counted leg link i -- j (i < j) between two chains    */
/*            whose refits have status 0: the circles m (above) of the two  */
/*            chains' refitted states at their heads, fused in the sense of  */
/*            i's chain: S = S_i + D S_j D, d = m_i - D m_j, x = m_i - S_i    */
/*            S^-1 d, C = S_i S^-1 D S_j D (symmetrised), chi2 = d^T S^-1 d  */
/*            (the joint circle of both legs for the linearised problem),    */
/*            written at i; elsewhere zeros and chi2 -1.                     */
/* ------------------------------------------------------------------------ */
#define REFIT_MAX_CHAIN 18
#define REFIT_NOT_HEAD 5
#define REFIT_LONG_CHAIN 6

static int next_link(int32_t i, int32_t n, const int32_t *next, const int32_t *prev, const int32_t *status)
{
    int32_t j = next[i];
    return j >= 0 && j < n && j != i && prev[j] == i && status[i] == 0 && status[j] == 0 ? j : -1;
}

static int prev_link(int32_t i, int32_t n, const int32_t *next, const int32_t *prev, const int32_t *status)
{
    int32_t a = prev[i];
    return a >= 0 && a < n && a != i && next[a] == i && status[i] == 0 && status[a] == 0 ? a : -1;
}

static int leg_link(int32_t i, int32_t n, const int32_t *leg, const int32_t *status)
{
    if (!leg) return -1;
    int32_t j = leg[i];
    return j >= 0 && j < n && j != i && leg[j] == i && status[i] == 0 && status[j] == 0 ? j : -1;
}

static int32_t uf_root(int32_t *p, int32_t x)
{
    while (p[x] != x) x = p[x];
    return x;
}

/* The head of i's chain (walking prev links), or -1 if there is none
 * within the chain length limit. */
static int32_t chain_head(int32_t i, int32_t n, const int32_t *next, const int32_t *prev, const int32_t *status)
{
    for (int32_t step = 0; step < REFIT_MAX_CHAIN; ++step) {
        int32_t a = prev_link(i, n, next, prev, status);
        if (a < 0) return i;
        i = a;
    }
    return -1;
}

static void refit_chain(int32_t head, int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                        const int32_t *sector, const int32_t *first_row, const int32_t *status,
                        const int32_t *next, const int32_t *prev, const double *y, const double *z,
                        const double *row_x, int32_t n_rows, int32_t n_sectors, const double *map,
                        const oracle_fit_params *prm, double *xo, double *po, double *co, double *chi2o,
                        int32_t *ndfo, int32_t *sto)
{
    int32_t segs[REFIT_MAX_CHAIN];
    int32_t ns = 0, n = 0, s = head;
    *xo = 0.0;
    *chi2o = 0.0;
    *ndfo = 0;
    for (int i = 0; i < 5; ++i) po[i] = 0.0;
    for (int i = 0; i < 15; ++i) co[i] = 0.0;
    while (s >= 0) {
        if (ns == REFIT_MAX_CHAIN) { *sto = REFIT_LONG_CHAIN; return; }
        segs[ns++] = s;
        n += offsets[s + 1] - offsets[s];
        s = next_link(s, n_tracks, next, prev, status);
    }
    *ndfo = 2 * n - 5;
    for (int q = 0; q < ns; ++q) {
        int32_t g = segs[q], m = offsets[g + 1] - offsets[g];
        if (m < 1 || first_row[g] < 0 || first_row[g] + m > n_rows || sector[g] < 0 || sector[g] >= n_sectors) {
            *sto = 1;
            return;
        }
    }
    /* the hit list: plane x, measurement and sector of each hit */
    double *hx = (double *)malloc(sizeof(double) * (size_t)n * 3);
    int32_t *hs = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * 2);
    double *hy = hx + n, *hz = hx + 2 * (size_t)n;
    int32_t *hg = hs + n;
    int32_t k = 0;
    for (int q = 0; q < ns; ++q) {
        int32_t g = segs[q], m = offsets[g + 1] - offsets[g];
        for (int32_t e = 0; e < m; ++e, ++k) {
            int32_t r = first_row[g] + e, c = hits[offsets[g] + e];
            hx[k] = row_x[r];
            hy[k] = y[c];
            hz[k] = z[c];
            if (map) {
                hy[k] -= map[((size_t)sector[g] * n_rows + r) * 2 + 0];
                hz[k] -= map[((size_t)sector[g] * n_rows + r) * 2 + 1];
            }
            hs[k] = sector[g];
            hg[k] = g;
        }
    }
    double p[5], C[25];
    int32_t st = 1;
    if (n >= 3) {
        /* the start: hits 0, (n-1)/2, n-1 in the frame of hit n-1 */
        int32_t idx[3] = {0, (n - 1) / 2, n - 1};
        double xs[3], ys[3], zs[3];
        double at = sector_angle(hs[n - 1], n_sectors);
        for (int q = 0; q < 3; ++q) {
            int32_t h = idx[q];
            double d = sector_angle(hs[h], n_sectors) - at;
            xs[q] = hx[h] * cos(d) - hy[h] * sin(d);
            ys[q] = hx[h] * sin(d) + hy[h] * cos(d);
            zs[q] = hz[h];
        }
        xs[2] = hx[n - 1];
        ys[2] = hy[n - 1];
        st = start_points(3, xs, ys, zs, prm, p, C);
    }
    double vy = prm->sigma_y * prm->sigma_y, vz = prm->sigma_z * prm->sigma_z;
    double chi2 = 0.0, xcur = hx[n - 1];
    for (k = n - 2; k >= 0 && !st; --k) {
        if (hg[k] == hg[k + 1]) {
            if (predict(p, C, hx[k] - hx[k + 1], prm)) { st = 2; break; }
        } else {
            double da = sector_angle(hs[k], n_sectors) - sector_angle(hs[k + 1], n_sectors);
            if (da > PI_D) da -= 2.0 * PI_D;
            if (da < -PI_D) da += 2.0 * PI_D;
            double pn[5], J[25], JC[25], Jt[25];
            if (oracle_transfer(p, hx[k + 1], da, hx[k], prm->bz, prm->max_sin, pn, J)) { st = 2; break; }
            mat5_mul(J, C, JC);
            for (int a = 0; a < 5; ++a)
                for (int b = 0; b < 5; ++b) Jt[a * 5 + b] = J[b * 5 + a];
            mat5_mul(JC, Jt, C);
            for (int a = 0; a < 5; ++a) p[a] = pn[a];
        }
        xcur = hx[k];
        if (update(p, C, hy[k], hz[k], vy, vz, &chi2)) { st = 3; break; }
    }
    if (n >= 3) {
        *xo = xcur;
        *chi2o = chi2;
        for (int i = 0; i < 5; ++i) po[i] = p[i];
        pack_cov(C, co);
    }
    *sto = st;
    free(hx);
    free(hs);
}

void oracle_refit(int32_t n_tracks, const int32_t *offsets, const int32_t *hits, const int32_t *sector,
                  const int32_t *first_row, const int32_t *status, const int32_t *next, const int32_t *prev,
                  const int32_t *leg, const double *y, const double *z, const double *row_x, int32_t n_rows,
                  int32_t n_sectors, const double *map, const oracle_fit_params *prm, int32_t *track_id,
                  double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *rstatus,
                  double *loop_par, double *loop_cov, double *loop_chi2)
{
    /* track ids: union of the linked segments, the smaller index the root */
    for (int32_t i = 0; i < n_tracks; ++i) track_id[i] = status[i] == 0 ? i : -1;
    for (int32_t i = 0; i < n_tracks; ++i) {
        int32_t nb[2] = {next_link(i, n_tracks, next, prev, status), leg_link(i, n_tracks, leg, status)};
        for (int e = 0; e < 2; ++e) {
            if (nb[e] < 0) continue;
            int32_t a = uf_root(track_id, i), b = uf_root(track_id, nb[e]);
            if (a < b) track_id[b] = a;
            else if (b < a) track_id[a] = b;
        }
    }
    for (int32_t i = 0; i < n_tracks; ++i)
        if (track_id[i] >= 0) track_id[i] = uf_root(track_id, i);
    /* chain refits at the heads */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n_tracks; ++i) {
        double *po = par + (size_t)i * 5, *co = cov + (size_t)i * 15;
        if (status[i] != 0 || prev_link(i, n_tracks, next, prev, status) >= 0) {
            x_out[i] = 0.0;
            chi2[i] = 0.0;
            ndf[i] = 0;
            rstatus[i] = REFIT_NOT_HEAD;
            for (int q = 0; q < 5; ++q) po[q] = 0.0;
            for (int q = 0; q < 15; ++q) co[q] = 0.0;
            continue;
        }
        refit_chain(i, n_tracks, offsets, hits, sector, first_row, status, next, prev, y, z, row_x, n_rows,
                    n_sectors, map, prm, &x_out[i], po, co, &chi2[i], &ndf[i], &rstatus[i]);
    }
    if (!loop_par) return;
    /* the joint circle of each pair of looper legs */
    for (int32_t i = 0; i < n_tracks; ++i) {
        double *lp = loop_par + (size_t)i * 4, *lc = loop_cov + (size_t)i * 10;
        for (int q = 0; q < 4; ++q) lp[q] = 0.0;
        for (int q = 0; q < 10; ++q) lc[q] = 0.0;
        loop_chi2[i] = -1.0;
        int32_t j = leg_link(i, n_tracks, leg, status);
        if (j <= i) continue;
        int32_t hi = chain_head(i, n_tracks, next, prev, status), hj = chain_head(j, n_tracks, next, prev, status);
        if (hi < 0 || hj < 0 || hi == hj || rstatus[hi] != 0 || rstatus[hj] != 0) continue;
        double mi[4], mj[4], Ji[20], Jj[20], Si[16], Sj[16], S[16], Sinv[16], d[4];
        if (oracle_leg_circle(par + (size_t)hi * 5, x_out[hi], sector_angle(sector[hi], n_sectors), prm->bz, mi, Ji) ||
            oracle_leg_circle(par + (size_t)hj * 5, x_out[hj], sector_angle(sector[hj], n_sectors), prm->bz, mj, Jj))
            continue;
        leg_cov(Ji, cov + (size_t)hi * 15, Si);
        leg_cov(Jj, cov + (size_t)hj * 15, Sj);
        /* D S_j D: the (centre, kappa/t) cross terms change sign */
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                Sj[a * 4 + b] *= ((a < 2) == (b < 2)) ? 1.0 : -1.0;
                S[a * 4 + b] = Si[a * 4 + b] + Sj[a * 4 + b];
            }
        d[0] = mi[0] - mj[0];
        d[1] = mi[1] - mj[1];
        d[2] = mi[2] + mj[2];
        d[3] = mi[3] + mj[3];
        if (inv4(S, Sinv)) continue;
        double K[16], Cf[16], chi = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double acc = 0.0;
                for (int q = 0; q < 4; ++q) acc += Si[a * 4 + q] * Sinv[q * 4 + b];
                K[a * 4 + b] = acc;                           /* S_i S^-1 */
            }
        for (int a = 0; a < 4; ++a) {
            double acc = mi[a];
            for (int q = 0; q < 4; ++q) acc -= K[a * 4 + q] * d[q];
            lp[a] = acc;
            for (int b = 0; b < 4; ++b) chi += d[a] * Sinv[a * 4 + b] * d[b];
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double acc = 0.0;
                for (int q = 0; q < 4; ++q) acc += K[a * 4 + q] * Sj[q * 4 + b];
                Cf[a * 4 + b] = acc;
            }
        for (int a = 0, q = 0; a < 4; ++a)
            for (int b = 0; b <= a; ++b, ++q) lc[q] = 0.5 * (Cf[a * 4 + b] + Cf[b * 4 + a]);
        loop_chi2[i] = chi;
    }
}
