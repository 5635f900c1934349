/* CPU oracle (test infrastructure only): declarations.  See tpc_oracle.c. */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H
#include <stdint.h>

typedef struct oracle_fit_params {
    double bz;          /* T */
    double sigma_y;     /* cm */
    double sigma_z;     /* cm */
    double max_sin;     /* |sin phi| limit */
    double var_sin0, var_tgl0, var_qpt0;   /* start covariance of s, t, w */
} oracle_fit_params;

typedef struct oracle_follow_params {
    double gate;        /* pickup gate on the predicted-residual chi2 (2 dof) */
    int32_t max_miss;   /* consecutive rows without pickup that are crossed */
} oracle_follow_params;

typedef struct oracle_material {
    double x0;          /* radiation length of the gas, cm (infinite: no scattering) */
    double mass;        /* mass hypothesis, GeV */
    double chi2_cut;    /* a hit whose predicted-residual chi2 exceeds this is not used */
    double rho;         /* density of the gas, g/cm^3 (0: no energy loss) */
    double z_over_a;    /* its Z/A, mol/g */
    double mean_exc;    /* its mean excitation energy I, GeV */
} oracle_material;

/* Mean energy loss <dE/dx> per density (GeV cm^2/g) of a unit-charge
 * particle of the given beta*gamma and mass (Bethe, no density effect). */
double oracle_bethe(double beta_gamma, double mass, double z_over_a, double mean_exc);

/* The energy-loss map of a segment of plane distance dx from state p
 * (dir +1: a step inwards, the loss given back; -1: outwards):
 * out = {w', dw'/dt, dw'/dw, straggling variance of w}.  Returns 1 if the
 * particle stops, else 0. */
int32_t oracle_eloss(const double *p, double dx, const oracle_material *m, double dir, double *out);

void oracle_set_threads(int n);
int oracle_max_threads(void);

void oracle_neighbours(int32_t n_segments, int32_t n_rows, const int32_t *row_offsets,
                       const float *y, const float *z, float win_y, float win_z,
                       float cut_y, float cut_z, int32_t *up, int32_t *dn);

int32_t oracle_ca_seed(int32_t n_segments, int32_t n_sectors, int32_t n_rows,
                       const int32_t *row_offsets, const int32_t *up, const int32_t *dn,
                       int32_t min_hits, int32_t cap_seeds, int32_t cap_hits,
                       int32_t *n_seeds_out, int32_t *n_hits_out, int32_t *offsets,
                       int32_t *hits, int32_t *frame, int32_t *sector, int32_t *first_row);

int32_t oracle_propagate(const double *p, double dx, double bz, double max_sin,
                         double *pout, double *F);

void oracle_fit(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                const int32_t *sector, const int32_t *first_row,
                const double *y, const double *z, const double *row_x, int32_t n_rows,
                const double *map, const oracle_fit_params *prm,
                double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                double *margin);

void oracle_follow(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                   const int32_t *frame, const int32_t *sector, const int32_t *first_row,
                   const int32_t *row_offsets, int32_t n_frames, int32_t n_sectors, int32_t n_rows,
                   const double *y, const double *z, const double *row_x,
                   const oracle_fit_params *prm, const oracle_follow_params *fp,
                   int32_t *rows, double *x_out, double *par, double *cov, double *chi2,
                   int32_t *ndf, int32_t *status, double *margin);

void oracle_fit_material(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                         const int32_t *first_row, const double *y, const double *z, const double *row_x,
                         const oracle_fit_params *prm, const oracle_material *mat,
                         double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                         uint8_t *rejected, double *margin);

void oracle_neighbours_skip(int32_t n_segments, int32_t n_rows, const int32_t *row_offsets,
                            const float *y, const float *z, float win_y, float win_z,
                            float cut_y, float cut_z, int32_t *up, int32_t *dn);

void oracle_fit_rows(int32_t n_tracks, const int32_t *offsets, const int32_t *hits,
                     const int32_t *frame, const int32_t *sector, const int32_t *row_offsets,
                     int32_t n_frames, int32_t n_sectors, int32_t n_rows,
                     const double *y, const double *z, const double *row_x, const float *err,
                     const oracle_fit_params *prm, const oracle_material *mat,
                     double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *status,
                     uint8_t *rejected, double *margin, double *hit_par, double *hit_cov);

/* rANS coder of integer arrays (rans_oracle.c) */
#include <stddef.h>
int64_t oracle_rans_freqs(const uint32_t *c, uint32_t R, uint64_t n, uint32_t L, uint32_t *f);
size_t oracle_rans_bound(int64_t n, uint32_t R, uint32_t B);
int32_t oracle_rans_encode(const int32_t *sym, int64_t n, uint32_t L, uint32_t B, uint32_t max_range,
                           uint8_t *out, size_t cap, size_t *size);
int32_t oracle_rans_decode(const uint8_t *in, size_t size, int32_t *out, int64_t cap, int64_t *n_out);
/* Cross-sector merging of fitted segments (see tpc_oracle.c): the transfer
 * of a state into a frame turned by da and on to plane xt (J may be NULL;
 * returns 0 or 2), and the mutual-best links between segments of
 * neighbouring sectors. */
int32_t oracle_transfer(const double *p, double x, double da, double xt, double bz, double max_sin,
                        double *pout, double *J);
void oracle_merge(int32_t n_tracks, const double *x, const double *par, const double *cov, const int32_t *status,
                  const int32_t *frame, const int32_t *sector, int32_t n_sectors, double bz, double max_sin,
                  double cut, int32_t *next, int32_t *prev, double *chi2, double *mpar, double *mcov);

/* Legs of loopers (see tpc_oracle.c): a segment's circle in global
 * coordinates m = (X_c, Y_c, kappa, tan lambda) with its 4x5 Jacobian (J may
 * be NULL; returns 1 for a circle too large or a degenerate state), and the
 * mutual-best pairing of legs. */
int32_t oracle_leg_circle(const double *p, double x, double alpha, double bz, double *m, double *J);
void oracle_legs(int32_t n_tracks, const double *x, const double *par, const double *cov, const int32_t *status,
                 const int32_t *frame, const int32_t *sector, int32_t n_sectors, double bz, double cut,
                 int32_t *leg, double *leg_chi2);

/* Tracks assembled from linked segments and refitted over all their hits
 * (see tpc_oracle.c): component ids, the refit of each chain at its head
 * (status 5 elsewhere, 6 for a chain of more than 18 segments) and the joint
 * circle of each pair of looper legs (leg and loop_* may be NULL). */
void oracle_refit(int32_t n_tracks, const int32_t *offsets, const int32_t *hits, const int32_t *sector,
                  const int32_t *first_row, const int32_t *status, const int32_t *next, const int32_t *prev,
                  const int32_t *leg, const double *y, const double *z, const double *row_x, int32_t n_rows,
                  int32_t n_sectors, const double *map, const oracle_fit_params *prm, int32_t *track_id,
                  double *x_out, double *par, double *cov, double *chi2, int32_t *ndf, int32_t *rstatus,
                  double *loop_par, double *loop_cov, double *loop_chi2);

void oracle_ctf_build(int32_t n_tracks, int32_t n_rows, int32_t n_sectors, int32_t n_segments,
                      const int32_t *row_offsets, const float *y, const float *z,
                      const int32_t *rows, const int32_t *status, const int32_t *frame,
                      const int32_t *sector, float qy, float qz, int32_t **arr, int64_t *count);
#endif
