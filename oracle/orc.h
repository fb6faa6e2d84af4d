/*
 * FP64 CPU oracle for the MS-GWaM-3D ray-volume hot path (Voelker et al.,
 * "MS-GWaM: A 3-dimensional transient gravity wave parametrization for
 * atmospheric models", arXiv 2309.11257).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  Only
 * the test-suite, the package smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or table with the GPU library.
 *
 * Plain, slow, obviously-correct C: one ray at a time, double precision
 * everywhere, no blocking or fusion, every expression evaluated left to right
 * as written (build with -ffp-contract=off, no fast-math).  Each function names
 * the passage of the paper it follows.
 *
 * Coordinates.  Cartesian: (x, y, z) in metres on a periodic f-plane box.
 * Spherical: (lambda, phi, z) = (longitude rad, latitude rad, height m) with
 * r = a + z.  The grid is cell-centred: centre i of a horizontal axis sits at
 * origin + (i + 1/2) d; level k sits at (k + 1/2) dz.
 *
 * Parity status (see the tests): every function is pinned by closed forms,
 * invariants, brute force or finite differences, except the merge pass, whose
 * invariants (wave action, pseudo-momentum, cell counts) are pinned but whose
 * choice of merge partners is a reading with no counterpart in the paper.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#define ORC_CARTESIAN 0
#define ORC_SPHERICAL 1

/* ray states */
#define ORC_ACTIVE 0
#define ORC_GONE_TOP 1
#define ORC_GONE_BOTTOM 2
#define ORC_GONE_POLE 3
#define ORC_INVALID 4
#define ORC_MERGED 5
#define ORC_CAPPED 6

typedef struct {
    int32_t geometry;
    int32_t nx, ny, nz;
    double dx, dy, dz;  /* m (Cartesian) or rad, rad, m (spherical) */
    double x0, y0;      /* horizontal origin: (0,0) Cartesian, (0,-pi/2) spherical */
    double a;           /* planetary radius, spherical only */
    /* resolved fields, cell centres, layout [nz][ny][nx] */
    const double *U, *V, *N2;
    const double *f2;   /* [ny]: Coriolis parameter squared per row */
    const double *rho;  /* [nz]: reference density per level */
    /* gradient fields filled by orc_prepare, same layout, per metre
       (Cartesian) or per radian (spherical horizontal) */
    double *Ux, *Uy, *Uz, *Vx, *Vy, *Vz, *N2x, *N2y, *N2z;
    double *f2y;        /* [ny] */
    const double *f;    /* [ny]: Coriolis parameter per row, signed */
    /* scale-height correction Gamma^2 at cell centres [nz][ny][nx]
       (Section 2a, eq. dispersion); NULL means Gamma = 0.  Its gradients are
       filled by orc_prepare when it is given. */
    const double *G2;
    double *G2x, *G2y, *G2z;
} orc_bg;

typedef struct {
    double *x, *y, *z, *k, *l, *m, *dx, *dy, *dz, *px, *py, *pz, *n;
    int64_t *id;
    uint8_t *state;  /* ORC_ACTIVE or the reason the ray left */
    int32_t *col;    /* column key j*nx+i after a step, -1 if not active */
} orc_rays;

typedef struct {
    int64_t n_active, n_top, n_bottom, n_pole, n_invalid, n_merged, n_capped, n_split;
    double sum_W, sum_kW, sum_lW, sum_mW, removed_W;
    int64_t n_launched;
    double launched_W;
} orc_tally;

/* continuous launch from a ghost layer (orc_launch) */
typedef struct {
    double z_launch;           /* top of the ghost layer: the launch height (m) */
    double dt;                 /* the step whose crossing the new volumes represent (s) */
    double t_solstice;         /* time since the northern summer solstice (s) */
    double F_s, F_w;           /* summer and winter launch fluxes of the latitudinal profile (Pa) */
    double lambda_h;           /* horizontal wavelength (m) */
    double c_min, c_max;       /* range of intrinsic horizontal phase speeds (m/s) */
    double c_center, c_width;  /* Gaussian spectral weight over the phase speeds */
    int32_t n_speeds;          /* phase-speed bins */
    const double *flux_col;    /* [ny*nx] launch flux per column (Pa), or NULL: the profile (sphere) */
} orc_launch_params;

void orc_prepare(orc_bg *g);
void orc_interp(const orc_bg *g, double x, double y, double z, double out[14]);
void orc_dispersion(double N2, double f2, double k, double l, double m, double out[4]);
void orc_dispersion_g(double N2, double f2, double G2, double k, double l, double m, double out[4]);
void orc_interp_gamma(const orc_bg *g, double x, double y, double z, double out[4]);
void orc_rhs(const orc_bg *g, const double Y[9], double F[9]);
void orc_step(const orc_bg *g, orc_rays *r, int64_t n, double dt, orc_tally *t);
void orc_keys(const orc_bg *g, orc_rays *r, int64_t n);
void orc_deposit(const orc_bg *g, const orc_rays *r, int64_t n, double *flux);
void orc_drag(const orc_bg *g, const double *flux, double *drag);
int64_t orc_split(const orc_bg *g, orc_rays *r, int64_t n, int64_t capacity,
                  double alpha, int64_t *next_id, orc_tally *t);
void orc_merge(const orc_bg *g, orc_rays *r, int64_t n, int32_t n_max, orc_tally *t);
void orc_cap(const orc_bg *g, orc_rays *r, int64_t n, int32_t n_max, orc_tally *t);
void orc_stats(const orc_rays *r, int64_t n, orc_tally *t);
void orc_features(const orc_bg *g, const orc_rays *r, int64_t n, double *X);
void orc_saturation(const orc_bg *g, orc_rays *r, int64_t n, double dt, double *P, double *Q, double *kappa,
                    int given_cols);
void orc_full_fluxes(const orc_bg *g, orc_rays *r, int64_t n, double *flux8, int given_cols);
void orc_smooth(const orc_bg *g, const double *in, int nslices, double *out);
void orc_divergence(const orc_bg *g, const double *Fx, const double *Fy, const double *Fz, double *out);
void orc_full_tendencies(const orc_bg *g, const double *flux8, double *out3);
void orc_budget(const orc_bg *g, orc_rays *r, int64_t n, double *fields4, int given_cols);
void orc_budget_terms(const orc_bg *g, const double *fields4, double *terms2);
double orc_launch_flux(const orc_bg *g, int j, const orc_launch_params *p);
int64_t orc_launch(const orc_bg *g, orc_rays *r, int64_t n, int64_t capacity, const orc_launch_params *p,
                   int64_t *next_id, orc_tally *t);
int orc_num_threads(void);
void orc_set_threads(int n);

#endif
