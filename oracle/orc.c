/*
 * FP64 CPU oracle for the MS-GWaM-3D ray-volume hot path.  TEST
 * INFRASTRUCTURE ONLY: see orc.h.  Build: gcc -O2 -std=c11 -ffp-contract=off
 * -fopenmp (no fast-math).  Every floating-point expression below is evaluated
 * in the order written.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(g, i, j, k) ((size_t)(k) * (size_t)(g)->ny * (size_t)(g)->nx + (size_t)(j) * (size_t)(g)->nx + (size_t)(i))

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Background preparation.  Section 3b: the mean fields *and their gradients*
 * are linearly interpolated to the ray-volume centre and faces.  The
 * gradients are formed once per background as centred differences
 * (chi[i+1] - chi[i-1]) / (2 d), periodic in x (and y on the Cartesian box),
 * one-sided at the vertical ends and, on the sphere, at the first and last
 * latitude rows.
 * ------------------------------------------------------------------------ */
static double ddx(const orc_bg *g, const double *F, int i, int j, int k)
{
    int ip = (i + 1) % g->nx, im = (i + g->nx - 1) % g->nx;
    return (F[IDX(g, ip, j, k)] - F[IDX(g, im, j, k)]) / (2.0 * g->dx);
}

static double ddy(const orc_bg *g, const double *F, int i, int j, int k)
{
    if (g->geometry == ORC_CARTESIAN) {
        int jp = (j + 1) % g->ny, jm = (j + g->ny - 1) % g->ny;
        return (F[IDX(g, i, jp, k)] - F[IDX(g, i, jm, k)]) / (2.0 * g->dy);
    }
    if (g->ny == 1) return 0.0;
    if (j == 0) return (F[IDX(g, i, 1, k)] - F[IDX(g, i, 0, k)]) / g->dy;
    if (j == g->ny - 1) return (F[IDX(g, i, j, k)] - F[IDX(g, i, j - 1, k)]) / g->dy;
    return (F[IDX(g, i, j + 1, k)] - F[IDX(g, i, j - 1, k)]) / (2.0 * g->dy);
}

static double ddz(const orc_bg *g, const double *F, int i, int j, int k)
{
    if (g->nz == 1) return 0.0;
    if (k == 0) return (F[IDX(g, i, j, 1)] - F[IDX(g, i, j, 0)]) / g->dz;
    if (k == g->nz - 1) return (F[IDX(g, i, j, k)] - F[IDX(g, i, j, k - 1)]) / g->dz;
    return (F[IDX(g, i, j, k + 1)] - F[IDX(g, i, j, k - 1)]) / (2.0 * g->dz);
}

void orc_prepare(orc_bg *g)
{
    int i, j, k;
    for (k = 0; k < g->nz; k++)
        for (j = 0; j < g->ny; j++)
            for (i = 0; i < g->nx; i++) {
                size_t c = IDX(g, i, j, k);
                g->Ux[c] = ddx(g, g->U, i, j, k);
                g->Uy[c] = ddy(g, g->U, i, j, k);
                g->Uz[c] = ddz(g, g->U, i, j, k);
                g->Vx[c] = ddx(g, g->V, i, j, k);
                g->Vy[c] = ddy(g, g->V, i, j, k);
                g->Vz[c] = ddz(g, g->V, i, j, k);
                g->N2x[c] = ddx(g, g->N2, i, j, k);
                g->N2y[c] = ddy(g, g->N2, i, j, k);
                g->N2z[c] = ddz(g, g->N2, i, j, k);
                if (g->G2) {
                    g->G2x[c] = ddx(g, g->G2, i, j, k);
                    g->G2y[c] = ddy(g, g->G2, i, j, k);
                    g->G2z[c] = ddz(g, g->G2, i, j, k);
                }
            }
    for (j = 0; j < g->ny; j++) {
        if (g->geometry == ORC_CARTESIAN) {
            int jp = (j + 1) % g->ny, jm = (j + g->ny - 1) % g->ny;
            g->f2y[j] = (g->f2[jp] - g->f2[jm]) / (2.0 * g->dy);
        } else if (g->ny == 1) {
            g->f2y[j] = 0.0;
        } else if (j == 0) {
            g->f2y[j] = (g->f2[1] - g->f2[0]) / g->dy;
        } else if (j == g->ny - 1) {
            g->f2y[j] = (g->f2[j] - g->f2[j - 1]) / g->dy;
        } else {
            g->f2y[j] = (g->f2[j + 1] - g->f2[j - 1]) / (2.0 * g->dy);
        }
    }
}

/* ------------------------------------------------------------------------
 * Linear interpolation (Appendix B, 3-D field interpolation).  On this
 * structured grid the horizontal Taylor expansion about the containing cell
 * is replaced by linear interpolation between the four surrounding cell
 * centres, and the vertical interpolation is linear between levels as in the
 * paper.  Position -> fractional index g = (p - origin)/d - 1/2.  Periodic
 * axes wrap the integer index; clamped axes (vertical, latitude) hold the
 * end value beyond the first and last centres.
 * ------------------------------------------------------------------------ */
static void axis_periodic(double p, double origin, double d, int n, int *i0, int *i1, double *w)
{
    double g = (p - origin) / d - 0.5;
    double fl;
    long long ii;
    if (!(fabs(g) < 1.0e15)) { /* non-finite or absurd: poison the weight */
        *i0 = 0;
        *i1 = 0;
        *w = g - g;
        return;
    }
    fl = floor(g);
    *w = g - fl;
    ii = (long long)fl % n;
    if (ii < 0) ii += n;
    *i0 = (int)ii;
    *i1 = (int)((ii + 1) % n);
}

static void axis_clamped(double p, double origin, double d, int n, int *i0, int *i1, double *w)
{
    double g = (p - origin) / d - 0.5;
    if (g != g) {
        *i0 = 0;
        *i1 = 0;
        *w = g;
        return;
    }
    if (g <= 0.0) {
        *i0 = 0;
        *i1 = 0;
        *w = 0.0;
    } else if (g >= (double)(n - 1)) {
        *i0 = n - 1;
        *i1 = n - 1;
        *w = 0.0;
    } else {
        double fl = floor(g);
        *i0 = (int)fl;
        *i1 = *i0 + 1;
        *w = g - fl;
    }
}

typedef struct {
    int i0, i1, j0, j1, k0, k1;
    double wx, wy, wz;
} corners;

static void locate(const orc_bg *g, double x, double y, double z, corners *c)
{
    axis_periodic(x, g->x0, g->dx, g->nx, &c->i0, &c->i1, &c->wx);
    if (g->geometry == ORC_CARTESIAN)
        axis_periodic(y, g->y0, g->dy, g->ny, &c->j0, &c->j1, &c->wy);
    else
        axis_clamped(y, g->y0, g->dy, g->ny, &c->j0, &c->j1, &c->wy);
    axis_clamped(z, 0.0, g->dz, g->nz, &c->k0, &c->k1, &c->wz);
}

/* lerp along x on four rows, then y on two, then z */
static double trilin(const orc_bg *g, const double *F, const corners *c)
{
    double a0 = F[IDX(g, c->i0, c->j0, c->k0)], a1 = F[IDX(g, c->i1, c->j0, c->k0)];
    double b0 = F[IDX(g, c->i0, c->j1, c->k0)], b1 = F[IDX(g, c->i1, c->j1, c->k0)];
    double d0 = F[IDX(g, c->i0, c->j0, c->k1)], d1 = F[IDX(g, c->i1, c->j0, c->k1)];
    double e0 = F[IDX(g, c->i0, c->j1, c->k1)], e1 = F[IDX(g, c->i1, c->j1, c->k1)];
    double c00 = a0 + c->wx * (a1 - a0);
    double c10 = b0 + c->wx * (b1 - b0);
    double c01 = d0 + c->wx * (d1 - d0);
    double c11 = e0 + c->wx * (e1 - e0);
    double c0 = c00 + c->wy * (c10 - c00);
    double c1 = c01 + c->wy * (c11 - c01);
    return c0 + c->wz * (c1 - c0);
}

static double rowlin(const double *F, const corners *c)
{
    return F[c->j0] + c->wy * (F[c->j1] - F[c->j0]);
}

/* out: U V N2 Ux Uy Uz Vx Vy Vz N2x N2y N2z f2 f2y */
void orc_interp(const orc_bg *g, double x, double y, double z, double out[14])
{
    corners c;
    locate(g, x, y, z, &c);
    out[0] = trilin(g, g->U, &c);
    out[1] = trilin(g, g->V, &c);
    out[2] = trilin(g, g->N2, &c);
    out[3] = trilin(g, g->Ux, &c);
    out[4] = trilin(g, g->Uy, &c);
    out[5] = trilin(g, g->Uz, &c);
    out[6] = trilin(g, g->Vx, &c);
    out[7] = trilin(g, g->Vy, &c);
    out[8] = trilin(g, g->Vz, &c);
    out[9] = trilin(g, g->N2x, &c);
    out[10] = trilin(g, g->N2y, &c);
    out[11] = trilin(g, g->N2z, &c);
    out[12] = rowlin(g->f2, &c);
    out[13] = rowlin(g->f2y, &c);
}

/* Gamma^2 and its gradients (x, y, z) at one point; all zero without Gamma */
void orc_interp_gamma(const orc_bg *g, double x, double y, double z, double out[4])
{
    corners c;
    if (!g->G2) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    locate(g, x, y, z, &c);
    out[0] = trilin(g, g->G2, &c);
    out[1] = trilin(g, g->G2x, &c);
    out[2] = trilin(g, g->G2y, &c);
    out[3] = trilin(g, g->G2z, &c);
}

/* U, V, N2, f2, Gamma^2 at one point (face evaluations) */
static void interp5(const orc_bg *g, double x, double y, double z, double *U, double *V, double *N2, double *f2,
                    double *G2)
{
    corners c;
    locate(g, x, y, z, &c);
    *U = trilin(g, g->U, &c);
    *V = trilin(g, g->V, &c);
    *N2 = trilin(g, g->N2, &c);
    *f2 = rowlin(g->f2, &c);
    *G2 = g->G2 ? trilin(g, g->G2, &c) : 0.0;
}

/* ------------------------------------------------------------------------
 * Dispersion relation (Section 2a, eq. dispersion) with the scale-height
 * correction and the positive intrinsic branch:
 *   omega_hat^2 = (N^2 kh^2 + f^2 (m^2 + Gamma^2)) / K^2,
 *   K^2 = kh^2 + m^2 + Gamma^2.
 * Intrinsic group velocity = gradient of omega_hat in wavenumber space
 * (eq. eikonal, right), written with
 *   N^2 - omega_hat^2 = (m^2 + Gamma^2)(N^2 - f^2)/K^2,
 *   omega_hat^2 - f^2 = kh^2 (N^2 - f^2)/K^2
 * so that no difference of nearly equal numbers is formed:
 *   cg_x = k (m^2 + Gamma^2)(N^2-f^2) / (omega_hat K^4),  cg_y likewise with l,
 *   cg_z = -m kh^2 (N^2-f^2) / (omega_hat K^4).
 * out: omega_hat, cg_x, cg_y, cg_z (intrinsic, i.e. without U).
 * orc_dispersion is the case Gamma = 0.
 * ------------------------------------------------------------------------ */
void orc_dispersion_g(double N2, double f2, double G2, double k, double l, double m, double out[4])
{
    double kh2 = k * k + l * l;
    double M2 = m * m + G2;
    double K2 = kh2 + M2;
    double K4 = K2 * K2;
    double om = sqrt((N2 * kh2 + f2 * M2) / K2);
    double d = N2 - f2;
    double den = om * K4;
    out[0] = om;
    out[1] = ((k * M2) * d) / den;
    out[2] = ((l * M2) * d) / den;
    out[3] = -(((m * kh2) * d) / den);
}

void orc_dispersion(double N2, double f2, double k, double l, double m, double out[4])
{
    orc_dispersion_g(N2, f2, 0.0, k, l, m, out);
}

/* the fields at a carrier (B as orc_interp) and the dispersion there */
static void disp_at(const orc_bg *g, double x, double y, double z, double k, double l, double m, double B[14],
                    double D[4], double *G2out)
{
    double G[4];
    orc_interp(g, x, y, z, B);
    orc_interp_gamma(g, x, y, z, G);
    orc_dispersion_g(B[2], B[12], G[0], k, l, m, D);
    if (G2out) *G2out = G[0];
}

/* ------------------------------------------------------------------------
 * Right-hand side of the ray-volume equations for one RK stage.
 * Y = (x, y, z, k, l, m, Dx, Dy, Dz), extents in coordinate units.
 *
 * Carrier wavenumber tendency (eq. eikonal-sphere 1-3; the Cartesian box is
 * its flat limit) from the fields and gradients at the centre, with
 *   d omega_hat / d N^2     = kh^2 / (2 omega_hat K^2),
 *   d omega_hat / d f^2     = (m^2 + Gamma^2) / (2 omega_hat K^2),
 *   d omega_hat / d Gamma^2 = -(kh^2 / (2 omega_hat K^2)) (N^2 - f^2) / K^2,
 * the bracketed sensitivities of the three equations.
 *
 * Carrier motion and extent rates (Section 3a and Appendix B): group
 * velocities at the centres of opposing faces, which carry the carrier's
 * wavevector but see the local background; their mean moves the carrier and
 * their difference is the rate of change of the extent.
 *
 * Spherical: face velocities (m/s) are converted to angular rates with
 * 1/(r cos phi) and 1/r; the metric terms use the carrier's own face-averaged
 * velocities (u_c, v_c, w_c).
 * ------------------------------------------------------------------------ */
/* ground-based group velocity along axis axn (0: x, 1: y, 2: z) of a volume
   with wavevector (k, l, m) at a face centre, from the background there */
static double face_velocity(const orc_bg *g, double x, double y, double z, double k, double l, double m, int axn)
{
    double Uf, Vf, N2f, f2f, G2f, D[4];
    interp5(g, x, y, z, &Uf, &Vf, &N2f, &f2f, &G2f);
    orc_dispersion_g(N2f, f2f, G2f, k, l, m, D);
    if (axn == 0) return Uf + D[1];
    if (axn == 1) return Vf + D[2];
    return D[3]; /* no vertical mean wind */
}

void orc_rhs(const orc_bg *g, const double Y[9], double F[9])
{
    double x = Y[0], y = Y[1], z = Y[2], k = Y[3], l = Y[4], m = Y[5];
    double Dx = Y[6], Dy = Y[7], Dz = Y[8];
    double kh2 = k * k + l * l;
    double B[14], G[4];
    double M2, K2, om, q, qf, qg;
    double cxp, cxm, cyp, cym, czp, czm;
    double gk, gl, gm;

    orc_interp(g, x, y, z, B);
    orc_interp_gamma(g, x, y, z, G);
    M2 = m * m + G[0];
    K2 = kh2 + M2;
    om = sqrt((B[2] * kh2 + B[12] * M2) / K2);
    q = kh2 / ((2.0 * om) * K2);
    qf = M2 / ((2.0 * om) * K2);
    qg = -((kh2 * (B[2] - B[12])) / (((2.0 * om) * K2) * K2));

    cxp = face_velocity(g, x + 0.5 * Dx, y, z, k, l, m, 0);
    cxm = face_velocity(g, x - 0.5 * Dx, y, z, k, l, m, 0);
    cyp = face_velocity(g, x, y + 0.5 * Dy, z, k, l, m, 1);
    cym = face_velocity(g, x, y - 0.5 * Dy, z, k, l, m, 1);
    czp = face_velocity(g, x, y, z + 0.5 * Dz, k, l, m, 2);
    czm = face_velocity(g, x, y, z - 0.5 * Dz, k, l, m, 2);

    /* refraction terms at the centre: B = U V N2 Ux Uy Uz Vx Vy Vz N2x N2y N2z f2 f2y,
       G = Gamma^2 and its x, y, z gradients */
    gk = (k * B[3] + l * B[6]) + q * B[9];
    gl = ((k * B[4] + l * B[7]) + q * B[10]) + qf * B[13];
    gm = (k * B[5] + l * B[8]) + q * B[11];
    if (g->G2) {
        gk = gk + qg * G[1];
        gl = gl + qg * G[2];
        gm = gm + qg * G[3];
    }

    if (g->geometry == ORC_CARTESIAN) {
        F[0] = 0.5 * (cxp + cxm);
        F[1] = 0.5 * (cyp + cym);
        F[2] = 0.5 * (czp + czm);
        F[3] = -gk;
        F[4] = -gl;
        F[5] = -gm;
        F[6] = cxp - cxm;
        F[7] = cyp - cym;
        F[8] = czp - czm;
    } else {
        double r = g->a + z;
        double cphi = cos(y);
        double tphi = tan(y);
        double rc = r * cphi;
        double uc = 0.5 * (cxp + cxm);
        double vc = 0.5 * (cyp + cym);
        double wc = 0.5 * (czp + czm);
        F[0] = uc / rc;
        F[1] = vc / r;
        F[2] = wc;
        F[3] = ((-gk) / rc - (k * wc) / r) + ((k * tphi) * vc) / r;
        F[4] = ((-gl) / r - (l * wc) / r) - ((k * tphi) * uc) / r;
        F[5] = ((-gm) + (k * uc) / r) + (l * vc) / r;
        F[6] = (cxp - cxm) / rc;
        F[7] = (cyp - cym) / r;
        F[8] = czp - czm;
    }
}

/* ------------------------------------------------------------------------
 * Low-storage three-stage Runge-Kutta scheme of Williamson (1980), as cited
 * in Appendix B (horizontal propagation and parallelization): for stages
 * s = 1..3,  Q <- A_s Q + dt F(Y),  Y <- Y + B_s Q,  with
 * A = (0, -5/9, -153/128) and B = (1/3, 15/16, 8/15).  The background is
 * held fixed over the step.
 * ------------------------------------------------------------------------ */
static void rk3(const orc_bg *g, double Y[9], double dt)
{
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double Bc[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    double Q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double F[9];
    int s, c;
    for (s = 0; s < 3; s++) {
        orc_rhs(g, Y, F);
        for (c = 0; c < 9; c++) {
            Q[c] = A[s] * Q[c] + dt * F[c];
            Y[c] = Y[c] + Bc[s] * Q[c];
        }
    }
}

static int column_of(const orc_bg *g, double x, double y)
{
    double fi = floor((x - g->x0) / g->dx);
    double fj = floor((y - g->y0) / g->dy);
    int i, j;
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(g->nx - 1)) fi = (double)(g->nx - 1);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(g->ny - 1)) fj = (double)(g->ny - 1);
    i = (int)fi;
    j = (int)fj;
    return j * g->nx + i;
}

/* periodic wrap into [origin, origin + L); returns 0 if the value is not
   within one period of the domain (a ray cannot move that far in a step) */
static int wrap(double *p, double origin, double L)
{
    double v = *p - origin;
    if (v < 0.0) {
        v = v + L;
        if (v >= L) v = 0.0;
    } else if (v >= L) {
        v = v - L;
    }
    if (!(v >= 0.0 && v < L)) return 0;
    *p = (origin == 0.0) ? v : v + origin;
    return 1;
}

/* ------------------------------------------------------------------------
 * Post-step bookkeeping after the RK3 update: validity, periodic wrap,
 * removal of rays that leave through the top or bottom (Section 3c discards
 * rays that leave the launch layer the wrong way; here the domain edges play
 * that role) or come within 0.5 degree of a pole (Section 2a: the pole is a
 * coordinate singularity), and the parent-column key (Appendix B: each ray
 * is associated with the column containing its carrier).
 * ------------------------------------------------------------------------ */
static uint8_t post_step(const orc_bg *g, double Y[9], int32_t *col)
{
    int c;
    double K2;
    for (c = 0; c < 9; c++)
        if (!isfinite(Y[c])) return ORC_INVALID;
    if (!(Y[6] > 0.0 && Y[7] > 0.0 && Y[8] > 0.0)) return ORC_INVALID;
    K2 = (Y[3] * Y[3] + Y[4] * Y[4]) + Y[5] * Y[5];
    if (K2 == 0.0) return ORC_INVALID;
    if (!wrap(&Y[0], g->x0, (double)g->nx * g->dx)) return ORC_INVALID;
    if (g->geometry == ORC_CARTESIAN) {
        if (!wrap(&Y[1], g->y0, (double)g->ny * g->dy)) return ORC_INVALID;
    } else {
        if (fabs(Y[1]) >= 89.5 * (3.14159265358979323846 / 180.0)) return ORC_GONE_POLE;
    }
    if (Y[2] < 0.0) return ORC_GONE_BOTTOM;
    if (Y[2] > (double)g->nz * g->dz) return ORC_GONE_TOP;
    *col = column_of(g, Y[0], Y[1]);
    return ORC_ACTIVE;
}

static double ray_W(const orc_rays *r, int64_t i)
{
    /* total wave action of the volume: N times the three phase-space areas */
    return ((r->n[i] * r->px[i]) * r->py[i]) * r->pz[i];
}

void orc_step(const orc_bg *g, orc_rays *r, int64_t n, double dt, orc_tally *t)
{
    int64_t i;
    uint8_t *before = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    memcpy(before, r->state, (size_t)n);
#pragma omp parallel for schedule(dynamic, 256)
    for (i = 0; i < n; i++) {
        double Y[9];
        int32_t col = -1;
        uint8_t st;
        if (r->state[i] != ORC_ACTIVE) continue;
        Y[0] = r->x[i];
        Y[1] = r->y[i];
        Y[2] = r->z[i];
        Y[3] = r->k[i];
        Y[4] = r->l[i];
        Y[5] = r->m[i];
        Y[6] = r->dx[i];
        Y[7] = r->dy[i];
        Y[8] = r->dz[i];
        rk3(g, Y, dt);
        st = post_step(g, Y, &col);
        r->x[i] = Y[0];
        r->y[i] = Y[1];
        r->z[i] = Y[2];
        r->k[i] = Y[3];
        r->l[i] = Y[4];
        r->m[i] = Y[5];
        r->dx[i] = Y[6];
        r->dy[i] = Y[7];
        r->dz[i] = Y[8];
        r->state[i] = st;
        r->col[i] = (st == ORC_ACTIVE) ? col : -1;
    }
    if (t) {
        for (i = 0; i < n; i++) {
            if (before[i] != ORC_ACTIVE || r->state[i] == ORC_ACTIVE) continue;
            switch (r->state[i]) {
            case ORC_GONE_TOP: t->n_top++; break;
            case ORC_GONE_BOTTOM: t->n_bottom++; break;
            case ORC_GONE_POLE: t->n_pole++; break;
            default: t->n_invalid++; break;
            }
            if (r->state[i] != ORC_INVALID) t->removed_W += ray_W(r, i);
        }
    }
    free(before);
}

void orc_keys(const orc_bg *g, orc_rays *r, int64_t n)
{
    int64_t i;
    for (i = 0; i < n; i++)
        r->col[i] = (r->state[i] == ORC_ACTIVE) ? column_of(g, r->x[i], r->y[i]) : -1;
}

/* ------------------------------------------------------------------------
 * Flux projection (Section 3b, Appendix A).  The mean-flow forcing uses the
 * pseudo-momentum flux, integral of cg_hat k_h N d^3k; a ray volume carries
 * W = N Px Py Pz of wave action (N times its wavenumber volume times its
 * physical volume), spread uniformly over its vertical extent.
 *  - Horizontal fluxes are cell averages over the ray volumes whose carrier
 *    lies in the column; the ray's share of level k is its overlap with
 *    [k dz, (k+1) dz] divided by its height.
 *  - Vertical fluxes live on level interfaces kk = 0..nz and integrate the
 *    ray volumes over the staggered cell [(kk-1/2) dz, (kk+1/2) dz] clipped
 *    to the domain.
 * Each value is divided by the cell volume.  flux layout:
 * [6][nz+1][ny][nx] = Fxk, Fxl, Fyk, Fyl (levels 0..nz-1; slot nz is 0),
 * Fzk, Fzl (interfaces 0..nz).  Order of summation: column ascending, then
 * ray index ascending, then level ascending.
 * ------------------------------------------------------------------------ */
static double cell_area(const orc_bg *g, int j, double zc)
{
    if (g->geometry == ORC_CARTESIAN) return g->dx * g->dy;
    {
        double r = g->a + zc;
        double phi = g->y0 + ((double)j + 0.5) * g->dy;
        return (((r * r) * cos(phi)) * g->dx) * g->dy;
    }
}

static void deposit_ray(const orc_bg *g, const orc_rays *r, int64_t i, int c, double *flux)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t colstride = (size_t)g->ny * (size_t)g->nx;
    int ci = c % g->nx, cj = c / g->nx;
    double B[14], D[4];
    double W = ray_W(r, i);
    double z = r->z[i], Dz = r->dz[i];
    double zb = z - 0.5 * Dz, zt = z + 0.5 * Dz;
    double Lz = (double)g->nz * g->dz;
    double k = r->k[i], l = r->l[i];
    int kk, klo, khi;

    disp_at(g, r->x[i], r->y[i], z, k, l, r->m[i], B, D, NULL);

    klo = (int)floor(zb / g->dz);
    khi = (int)floor(zt / g->dz);
    if (klo < 0) klo = 0;
    if (khi > g->nz - 1) khi = g->nz - 1;
    for (kk = klo; kk <= khi; kk++) {
        double lo = (double)kk * g->dz, hi = (double)(kk + 1) * g->dz;
        double o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        double frac, vol;
        size_t at;
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, ((double)kk + 0.5) * g->dz) * g->dz;
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        flux[0 * plane + at] += (((D[1] * k) * W) * frac) / vol;
        flux[1 * plane + at] += (((D[1] * l) * W) * frac) / vol;
        flux[2 * plane + at] += (((D[2] * k) * W) * frac) / vol;
        flux[3 * plane + at] += (((D[2] * l) * W) * frac) / vol;
    }
    klo = (int)floor(zb / g->dz + 0.5);
    khi = (int)floor(zt / g->dz + 0.5);
    if (klo < 0) klo = 0;
    if (khi > g->nz) khi = g->nz;
    for (kk = klo; kk <= khi; kk++) {
        double lo = ((double)kk - 0.5) * g->dz, hi = ((double)kk + 0.5) * g->dz;
        double o, frac, vol;
        size_t at;
        if (lo < 0.0) lo = 0.0;
        if (hi > Lz) hi = Lz;
        o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, (double)kk * g->dz) * (hi - lo);
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        flux[4 * plane + at] += (((D[3] * k) * W) * frac) / vol;
        flux[5 * plane + at] += (((D[3] * l) * W) * frac) / vol;
    }
}

void orc_deposit(const orc_bg *g, const orc_rays *r, int64_t n, double *flux)
{
    int ncol = g->nx * g->ny;
    size_t total = (size_t)6 * (size_t)(g->nz + 1) * (size_t)ncol;
    int64_t *start = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t i;
    int c;
    memset(flux, 0, total * sizeof(double));
    /* stable counting sort of active rays by column key */
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) start[r->col[i] + 1]++;
    for (c = 0; c < ncol; c++) start[c + 1] += start[c];
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) {
            int cc = r->col[i];
            order[start[cc] + fill[cc]] = i;
            fill[cc]++;
        }
#pragma omp parallel for schedule(dynamic, 16)
    for (c = 0; c < ncol; c++) {
        int64_t p;
        for (p = start[c]; p < start[c + 1]; p++) deposit_ray(g, r, order[p], c, flux);
    }
    free(start);
    free(fill);
    free(order);
}

/* ------------------------------------------------------------------------
 * Drag (eq. mean-flow-impact with the pseudo-momentum approximation):
 * du = -(1/rho) div(Fk), dv = -(1/rho) div(Fl), centred differences of the
 * cell-mean horizontal fluxes (periodic, one-sided at the latitude ends) and
 * the difference of the interface fluxes across the level.  On the sphere
 * the horizontal divergence is (1/(r cos phi)) [d_lambda Fx + d_phi (cos phi
 * Fy)] with r = a + z_k; further metric terms of the tensor divergence are
 * left out.  drag layout [2][nz][ny][nx].
 * ------------------------------------------------------------------------ */
void orc_drag(const orc_bg *g, const double *flux, double *drag)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t cells = (size_t)g->nz * (size_t)g->ny * (size_t)g->nx;
    size_t at;
    int comp;
    for (comp = 0; comp < 2; comp++) {
        double *out = drag + (size_t)comp * cells;
        orc_divergence(g, flux + (size_t)(0 + comp) * plane, flux + (size_t)(2 + comp) * plane,
                       flux + (size_t)(4 + comp) * plane, out);
        for (at = 0; at < cells; at++) {
            int k = (int)(at / ((size_t)g->ny * (size_t)g->nx));
            out[at] = -(out[at] / g->rho[k]);
        }
    }
}

/* ------------------------------------------------------------------------
 * Vertical splitting (Appendix B, ray volume splitting): a volume taller
 * than alpha dz is cut into two equal halves with the same wavevector and
 * wave-action density, carriers at the half centres z -/+ Dz/4, heights
 * Dz/2 and vertical phase-space areas Pz/2; repeated until no piece exceeds
 * the threshold.  The lowest piece keeps the slot and id; the others are
 * appended in order of parent index and then height, with consecutive new
 * ids.  Returns the new count, or -1 (nothing changed) if capacity is short.
 * (The paper's floor of 1 km on the threshold is left to the caller's alpha.)
 * ------------------------------------------------------------------------ */
int64_t orc_split(const orc_bg *g, orc_rays *r, int64_t n, int64_t capacity,
                  double alpha, int64_t *next_id, orc_tally *t)
{
    double thr = alpha * g->dz;
    int64_t extra = 0, i, out = n;
    for (i = 0; i < n; i++) {
        double D = r->dz[i];
        int64_t pieces = 1;
        if (r->state[i] != ORC_ACTIVE) continue;
        while (D > thr && pieces < 64) {
            D = 0.5 * D;
            pieces *= 2;
        }
        extra += pieces - 1;
    }
    if (n + extra > capacity) return -1;
    for (i = 0; i < n; i++) {
        double zs[64], Ds[64], Ps[64];
        int np = 1, p;
        if (r->state[i] != ORC_ACTIVE || !(r->dz[i] > thr)) continue;
        zs[0] = r->z[i];
        Ds[0] = r->dz[i];
        Ps[0] = r->pz[i];
        while (Ds[0] > thr && np < 64) {
            double nz_[64], nD[64], nP[64];
            for (p = 0; p < np; p++) {
                nz_[2 * p] = zs[p] - 0.25 * Ds[p];
                nz_[2 * p + 1] = zs[p] + 0.25 * Ds[p];
                nD[2 * p] = 0.5 * Ds[p];
                nD[2 * p + 1] = 0.5 * Ds[p];
                nP[2 * p] = 0.5 * Ps[p];
                nP[2 * p + 1] = 0.5 * Ps[p];
            }
            np *= 2;
            memcpy(zs, nz_, sizeof(double) * (size_t)np);
            memcpy(Ds, nD, sizeof(double) * (size_t)np);
            memcpy(Ps, nP, sizeof(double) * (size_t)np);
        }
        for (p = 1; p < np; p++) {
            int64_t o = out++;
            r->x[o] = r->x[i];
            r->y[o] = r->y[i];
            r->z[o] = zs[p];
            r->k[o] = r->k[i];
            r->l[o] = r->l[i];
            r->m[o] = r->m[i];
            r->dx[o] = r->dx[i];
            r->dy[o] = r->dy[i];
            r->dz[o] = Ds[p];
            r->px[o] = r->px[i];
            r->py[o] = r->py[i];
            r->pz[o] = Ps[p];
            r->n[o] = r->n[i];
            r->id[o] = (*next_id)++;
            r->state[o] = ORC_ACTIVE;
            r->col[o] = r->col[i];
        }
        r->z[i] = zs[0];
        r->dz[i] = Ds[0];
        r->pz[i] = Ps[0];
        if (t) t->n_split += np - 1;
    }
    return out;
}

/* ------------------------------------------------------------------------
 * Per-cell merge (a reading: the paper caps ray counts per column, see
 * orc_cap; this pass instead merges ray volumes in any 3-D cell holding more
 * than n_max of them).  The cell's rays are ordered by spectral group
 * (azimuth octant of (k,l), sign of m, binary exponent of |m|) and then id;
 * one pass walks the order and merges adjacent pairs of the same group,
 * stopping once the count is n_max; if a pass finds no such pair, adjacent
 * pairs are merged regardless of group.  A merged volume keeps the first
 * ray's slot and id, the summed wave action W, W-weighted carrier position
 * and wavevector (conserving the pseudo-momentum sums), physical and spectral
 * extents spanning both volumes, phase-space areas recomputed from those
 * extents, and N = W / (Px Py Pz).
 * ------------------------------------------------------------------------ */
static int octant(double k, double l)
{
    int q = (k >= 0.0) ? (l >= 0.0 ? 0 : 3) : (l >= 0.0 ? 1 : 2);
    int big_l = fabs(l) > fabs(k);
    int off = (q == 0 || q == 2) ? big_l : !big_l;
    return 2 * q + off;
}

static int64_t group_key(double k, double l, double m)
{
    int e;
    frexp(fabs(m), &e);
    return ((int64_t)(octant(k, l) * 2 + (m < 0.0 ? 0 : 1)) << 16) + (int64_t)(e + 4096);
}

typedef struct {
    int64_t grp, id, idx;
} mrec;

static int mrec_cmp(const void *a, const void *b)
{
    const mrec *x = (const mrec *)a, *y = (const mrec *)b;
    if (x->grp != y->grp) return x->grp < y->grp ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static double metric_x(const orc_bg *g, double y, double z, double D)
{
    if (g->geometry == ORC_CARTESIAN) return D;
    return ((g->a + z) * cos(y)) * D;
}

static double metric_y(const orc_bg *g, double z, double D)
{
    if (g->geometry == ORC_CARTESIAN) return D;
    return (g->a + z) * D;
}

static void merge_pair(const orc_bg *g, orc_rays *r, int64_t a, int64_t b)
{
    double Wa = ray_W(r, a), Wb = ray_W(r, b), W = Wa + Wb;
    /* spectral extents before the merge */
    double dka = r->px[a] / metric_x(g, r->y[a], r->z[a], r->dx[a]);
    double dkb = r->px[b] / metric_x(g, r->y[b], r->z[b], r->dx[b]);
    double dla = r->py[a] / metric_y(g, r->z[a], r->dy[a]);
    double dlb = r->py[b] / metric_y(g, r->z[b], r->dy[b]);
    double dma = r->pz[a] / r->dz[a], dmb = r->pz[b] / r->dz[b];
    double lo, hi, x, y, z, k, l, m, Dx, Dy, Dz, Dk, Dl, Dm;
#define HULL(ca, da, cb, db, OUTD)                                            \
    do {                                                                      \
        double la_ = (ca) - 0.5 * (da), lb_ = (cb) - 0.5 * (db);              \
        double ha_ = (ca) + 0.5 * (da), hb_ = (cb) + 0.5 * (db);              \
        lo = la_ < lb_ ? la_ : lb_;                                           \
        hi = ha_ > hb_ ? ha_ : hb_;                                           \
        OUTD = hi - lo;                                                       \
    } while (0)
    x = (r->x[a] * Wa + r->x[b] * Wb) / W;
    y = (r->y[a] * Wa + r->y[b] * Wb) / W;
    z = (r->z[a] * Wa + r->z[b] * Wb) / W;
    k = (r->k[a] * Wa + r->k[b] * Wb) / W;
    l = (r->l[a] * Wa + r->l[b] * Wb) / W;
    m = (r->m[a] * Wa + r->m[b] * Wb) / W;
    HULL(r->x[a], r->dx[a], r->x[b], r->dx[b], Dx);
    HULL(r->y[a], r->dy[a], r->y[b], r->dy[b], Dy);
    HULL(r->z[a], r->dz[a], r->z[b], r->dz[b], Dz);
    HULL(r->k[a], dka, r->k[b], dkb, Dk);
    HULL(r->l[a], dla, r->l[b], dlb, Dl);
    HULL(r->m[a], dma, r->m[b], dmb, Dm);
#undef HULL
    (void)lo;
    (void)hi;
    r->x[a] = x;
    r->y[a] = y;
    r->z[a] = z;
    r->k[a] = k;
    r->l[a] = l;
    r->m[a] = m;
    r->dx[a] = Dx;
    r->dy[a] = Dy;
    r->dz[a] = Dz;
    r->px[a] = metric_x(g, y, z, Dx) * Dk;
    r->py[a] = metric_y(g, z, Dy) * Dl;
    r->pz[a] = Dz * Dm;
    r->n[a] = W / ((r->px[a] * r->py[a]) * r->pz[a]);
}

static int level_of(const orc_bg *g, double z)
{
    double fk = floor(z / g->dz);
    if (fk < 0.0) fk = 0.0;
    if (fk > (double)(g->nz - 1)) fk = (double)(g->nz - 1);
    return (int)fk;
}

void orc_merge(const orc_bg *g, orc_rays *r, int64_t n, int32_t n_max, orc_tally *t)
{
    int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
    int64_t *cnt = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *start, *order, i;
    int64_t c;
    orc_keys(g, r, n);
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) cnt[(int64_t)r->col[i] * g->nz + level_of(g, r->z[i]) + 1]++;
    start = cnt;
    for (c = 0; c < ncell; c++) start[c + 1] += start[c];
    order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(start[ncell] > 0 ? start[ncell] : 1));
    {
        int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
        for (i = 0; i < n; i++)
            if (r->state[i] == ORC_ACTIVE) {
                int64_t cc = (int64_t)r->col[i] * g->nz + level_of(g, r->z[i]);
                order[start[cc] + fill[cc]++] = i;
            }
        free(fill);
    }
    for (c = 0; c < ncell; c++) {
        int64_t len = start[c + 1] - start[c], count = len, p;
        mrec *rec;
        if (len <= n_max) continue;
        rec = (mrec *)malloc(sizeof(mrec) * (size_t)len);
        while (count > n_max) {
            int64_t m_ = 0, merged = 0, q;
            for (p = 0; p < len; p++) {
                int64_t idx = order[start[c] + p];
                if (r->state[idx] != ORC_ACTIVE) continue;
                rec[m_].grp = group_key(r->k[idx], r->l[idx], r->m[idx]);
                rec[m_].id = r->id[idx];
                rec[m_].idx = idx;
                m_++;
            }
            qsort(rec, (size_t)m_, sizeof(mrec), mrec_cmp);
            for (q = 0; q + 1 < m_ && count > n_max;) {
                if (rec[q].grp == rec[q + 1].grp) {
                    merge_pair(g, r, rec[q].idx, rec[q + 1].idx);
                    r->state[rec[q + 1].idx] = ORC_MERGED;
                    count--;
                    merged++;
                    q += 2;
                } else {
                    q += 1;
                }
            }
            if (merged == 0) {
                for (q = 0; q + 1 < m_ && count > n_max; q += 2) {
                    merge_pair(g, r, rec[q].idx, rec[q + 1].idx);
                    r->state[rec[q + 1].idx] = ORC_MERGED;
                    count--;
                    merged++;
                }
            }
            if (t) t->n_merged += merged;
        }
        free(rec);
    }
    /* merged carriers stay within their cell; refresh keys anyway */
    for (i = 0; i < n; i++) {
        if (r->state[i] != ORC_ACTIVE) {
            r->col[i] = -1;
            continue;
        }
        if (!wrap(&r->x[i], g->x0, (double)g->nx * g->dx) ||
            (g->geometry == ORC_CARTESIAN && !wrap(&r->y[i], g->y0, (double)g->ny * g->dy))) {
            r->state[i] = ORC_INVALID;
            r->col[i] = -1;
            continue;
        }
        r->col[i] = column_of(g, r->x[i], r->y[i]);
    }
    free(cnt);
    free(order);
}

/* ------------------------------------------------------------------------
 * Per-column cap (Appendix B, computational performance): a column holding
 * more than n_max ray volumes loses the ones with the lowest wave energy
 * E = omega_hat W (omega_hat at the carrier); among equal energies the larger
 * id goes first.
 * ------------------------------------------------------------------------ */
typedef struct {
    double E;
    int64_t id, idx;
} crec;

static int crec_cmp(const void *a, const void *b)
{
    const crec *x = (const crec *)a, *y = (const crec *)b;
    if (x->E != y->E) return x->E < y->E ? -1 : 1;
    if (x->id != y->id) return x->id > y->id ? -1 : 1;
    return 0;
}

void orc_cap(const orc_bg *g, orc_rays *r, int64_t n, int32_t n_max, orc_tally *t)
{
    int ncol = g->nx * g->ny;
    int64_t *start = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)ncol, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *hit = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t i;
    int c;
    orc_keys(g, r, n);
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) start[r->col[i] + 1]++;
    for (c = 0; c < ncol; c++) start[c + 1] += start[c];
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) order[start[r->col[i]] + fill[r->col[i]]++] = i;
    for (c = 0; c < ncol; c++) {
        int64_t len = start[c + 1] - start[c], p;
        crec *rec;
        if (len <= n_max) continue;
        rec = (crec *)malloc(sizeof(crec) * (size_t)len);
        for (p = 0; p < len; p++) {
            int64_t idx = order[start[c] + p];
            double B[14], D[4];
            disp_at(g, r->x[idx], r->y[idx], r->z[idx], r->k[idx], r->l[idx], r->m[idx], B, D, NULL);
            rec[p].E = D[0] * ray_W(r, idx);
            rec[p].id = r->id[idx];
            rec[p].idx = idx;
        }
        qsort(rec, (size_t)len, sizeof(crec), crec_cmp);
        for (p = 0; p < len - n_max; p++) {
            r->state[rec[p].idx] = ORC_CAPPED;
            r->col[rec[p].idx] = -1;
            hit[rec[p].idx] = 1;
        }
        free(rec);
    }
    if (t) {
        for (i = 0; i < n; i++)
            if (hit[i]) {
                t->n_capped++;
                t->removed_W += ray_W(r, i);
            }
    }
    free(hit);
    free(start);
    free(fill);
    free(order);
}

/* Diagnostics: wave action and pseudo-momentum sums over active rays in
   array order (the conserved quantities of Section 2a without sources). */
void orc_stats(const orc_rays *r, int64_t n, orc_tally *t)
{
    int64_t i;
    t->n_active = 0;
    t->sum_W = t->sum_kW = t->sum_lW = t->sum_mW = 0.0;
    for (i = 0; i < n; i++) {
        double W;
        if (r->state[i] != ORC_ACTIVE) continue;
        W = ray_W(r, i);
        t->n_active++;
        t->sum_W += W;
        t->sum_kW += r->k[i] * W;
        t->sum_lW += r->l[i] * W;
        t->sum_mW += r->m[i] * W;
    }
}

/* ------------------------------------------------------------------------
 * Column features of the surrogate (no counterpart in the paper; they
 * summarise the ray-volume state that the flux projection of Section 3b
 * reads).  Row c = j*nx + i of X [ncol][3*nz + 48]:
 *   U, V, N2 at the column's cell centres, levels 0..nz-1;
 *   for each of 8 azimuth sectors s (centred on the directions s*45 degrees
 *   of the horizontal wavevector, boundaries at 22.5 + 45 n degrees), six
 *   moments: sum W, sum |cg_z| k_h W, and the W-weighted means of log10 k_h,
 *   log10 |m| and the carrier height z, and the W-weighted standard deviation
 *   of z (sqrt of mean z^2 - mean^2, floored at 0); the means and the
 *   deviation are 0 for an empty sector;
 * over the active rays whose carrier lies in the column (col[] must hold the
 * keys), summed in ascending index.  cg_z is the intrinsic vertical group
 * velocity at the carrier (Section 2a), W = N Px Py Pz the wave action of
 * the volume (Section 3a).
 * The sector test compares |l| with tan(22.5 deg) |k| and vice versa, so no
 * arctangent decides an integer.
 * ------------------------------------------------------------------------ */
static int azimuth_sector(double k, double l)
{
    const double t = 0.41421356237309503; /* tan(pi/8) = sqrt(2) - 1 */
    double ak = fabs(k), al = fabs(l);
    if (al <= t * ak) return k > 0.0 ? 0 : 4;
    if (ak <= t * al) return l > 0.0 ? 2 : 6;
    if (k > 0.0) return l > 0.0 ? 1 : 7;
    return l > 0.0 ? 3 : 5;
}

void orc_features(const orc_bg *g, const orc_rays *r, int64_t n, double *X)
{
    int ncol = g->nx * g->ny, nf = 3 * g->nz + 48;
    int c, k, s;
    int64_t i;
    memset(X, 0, sizeof(double) * (size_t)ncol * (size_t)nf);
    for (c = 0; c < ncol; c++) {
        int ci = c % g->nx, cj = c / g->nx;
        double *row = X + (size_t)c * (size_t)nf;
        for (k = 0; k < g->nz; k++) {
            row[k] = g->U[IDX(g, ci, cj, k)];
            row[g->nz + k] = g->V[IDX(g, ci, cj, k)];
            row[2 * g->nz + k] = g->N2[IDX(g, ci, cj, k)];
        }
    }
    for (i = 0; i < n; i++) {
        double B[14], D[4], W, kh, z, *mom;
        if (r->state[i] != ORC_ACTIVE) continue;
        disp_at(g, r->x[i], r->y[i], r->z[i], r->k[i], r->l[i], r->m[i], B, D, NULL);
        W = ray_W(r, i);
        kh = sqrt(r->k[i] * r->k[i] + r->l[i] * r->l[i]);
        z = r->z[i];
        s = azimuth_sector(r->k[i], r->l[i]);
        mom = X + (size_t)r->col[i] * (size_t)nf + 3 * g->nz + 6 * s;
        mom[0] += W;
        mom[1] += fabs(D[3]) * kh * W;
        mom[2] += W * log10(kh);
        mom[3] += W * log10(fabs(r->m[i]));
        mom[4] += W * z;
        mom[5] += W * z * z;
    }
    for (c = 0; c < ncol; c++)
        for (s = 0; s < 8; s++) {
            double *mom = X + (size_t)c * (size_t)nf + 3 * g->nz + 6 * s;
            if (mom[0] > 0.0) {
                double zm, var;
                mom[2] = mom[2] / mom[0];
                mom[3] = mom[3] / mom[0];
                zm = mom[4] / mom[0];
                var = mom[5] / mom[0] - zm * zm;
                mom[4] = zm;
                mom[5] = var > 0.0 ? sqrt(var) : 0.0;
            } else {
                mom[2] = 0.0;
                mom[3] = 0.0;
                mom[4] = 0.0;
                mom[5] = 0.0;
            }
        }
}

/* ------------------------------------------------------------------------
 * Spectral saturation (Section 3c, eq. instability-threshold and
 * eq. turbulent-diffusivity).  Static instability is judged per grid cell
 * from the spectrally integrated quantity
 *   P = sum_j P_j,  P_j = (m^2 kh^2 / (omega_hat K^2)) A_j alpha_j,
 * with A_j = N_j dk dl dm the volume's wave action per unit physical volume
 * and alpha_j the fraction of the cell's volume the ray volume fills.  With
 * the projection of the fluxes (the whole volume in its carrier's column,
 * spread uniformly over its height) A_j alpha_j for level k is
 *   W_j (o_jk / Dz_j) / (A_c dz),  W_j = N_j Px Py Pz,
 * o_jk the overlap of [z - Dz/2, z + Dz/2] with the level.  omega_hat and K
 * are those of the carrier, K^2 = kh^2 + m^2 + Gamma^2 as the dispersion
 * relation defines it.  Where P exceeds rho_k / 2 the
 * turbulent diffusivity
 *   kappa = max(0, (P - rho/2) / (2 dt sum_j P_j K_j^2))
 * damps every volume there: N_j <- N_j (1 - 2 kappa K_j^2 dt).  A volume
 * that covers several levels takes the overlap-weighted mean of kappa over
 * them (levels outside the domain contribute nothing); the factor is held at
 * 0 or above, so that N never turns negative (the paper's argument that it
 * stays positive assumes the excess built up over one step).
 * Outputs P, Q = sum_j P_j K_j^2 and kappa on [nz][ny][nx]; the densities of
 * the active volumes are updated in place.  With given_cols the column keys
 * already in r->col are used (the parity tests hand in a lower-precision
 * path's decision for a volume at a cell face), else they are computed.  Order of summation as in
 * orc_deposit: column ascending, ray index ascending, level ascending.
 * ------------------------------------------------------------------------ */
static double saturation_weight(const orc_bg *g, const orc_rays *r, int64_t i, double *K2out)
{
    double B[14], D[4], G2;
    double k = r->k[i], l = r->l[i], m = r->m[i];
    double kh2 = k * k + l * l;
    double m2 = m * m;
    double K2;
    disp_at(g, r->x[i], r->y[i], r->z[i], k, l, m, B, D, &G2);
    K2 = kh2 + (m2 + G2);
    *K2out = K2;
    return (m2 * kh2) / (D[0] * K2);
}

void orc_saturation(const orc_bg *g, orc_rays *r, int64_t n, double dt, double *P, double *Q, double *kappa,
                    int given_cols)
{
    int ncol = g->nx * g->ny;
    size_t cells = (size_t)g->nz * (size_t)ncol;
    int64_t *start = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t i;
    int c;
    if (!given_cols) orc_keys(g, r, n);
    memset(P, 0, cells * sizeof(double));
    memset(Q, 0, cells * sizeof(double));
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) start[r->col[i] + 1]++;
    for (c = 0; c < ncol; c++) start[c + 1] += start[c];
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) {
            int cc = r->col[i];
            order[start[cc] + fill[cc]] = i;
            fill[cc]++;
        }
    /* per-cell sums */
#pragma omp parallel for schedule(dynamic, 16)
    for (c = 0; c < ncol; c++) {
        int ci = c % g->nx, cj = c / g->nx;
        int64_t p;
        for (p = start[c]; p < start[c + 1]; p++) {
            int64_t j = order[p];
            double K2;
            double s = saturation_weight(g, r, j, &K2);
            double W = ray_W(r, j);
            double zb = r->z[j] - 0.5 * r->dz[j], zt = r->z[j] + 0.5 * r->dz[j];
            int kk, klo = (int)floor(zb / g->dz), khi = (int)floor(zt / g->dz);
            if (klo < 0) klo = 0;
            if (khi > g->nz - 1) khi = g->nz - 1;
            for (kk = klo; kk <= khi; kk++) {
                double lo = (double)kk * g->dz, hi = (double)(kk + 1) * g->dz;
                double o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
                double vol, aw;
                size_t at;
                if (!(o > 0.0)) continue;
                vol = cell_area(g, cj, ((double)kk + 0.5) * g->dz) * g->dz;
                aw = (W * (o / r->dz[j])) / vol;
                at = IDX(g, ci, cj, kk);
                P[at] += s * aw;
                Q[at] += (s * K2) * aw;
            }
        }
    }
    /* turbulent diffusivity per cell */
    {
        size_t at;
        for (at = 0; at < cells; at++) {
            int kk = (int)(at / (size_t)ncol);
            double ex = P[at] - 0.5 * g->rho[kk];
            kappa[at] = (ex > 0.0 && Q[at] > 0.0) ? ex / ((2.0 * dt) * Q[at]) : 0.0;
        }
    }
    /* damping of every active volume by its overlap-weighted kappa */
#pragma omp parallel for schedule(dynamic, 256)
    for (i = 0; i < n; i++) {
        int ci, cj, kk, klo, khi;
        double zb, zt, kbar = 0.0, K2, fac;
        if (r->state[i] != ORC_ACTIVE) continue;
        ci = r->col[i] % g->nx;
        cj = r->col[i] / g->nx;
        zb = r->z[i] - 0.5 * r->dz[i];
        zt = r->z[i] + 0.5 * r->dz[i];
        klo = (int)floor(zb / g->dz);
        khi = (int)floor(zt / g->dz);
        if (klo < 0) klo = 0;
        if (khi > g->nz - 1) khi = g->nz - 1;
        for (kk = klo; kk <= khi; kk++) {
            double lo = (double)kk * g->dz, hi = (double)(kk + 1) * g->dz;
            double o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
            if (!(o > 0.0)) continue;
            kbar += (o / r->dz[i]) * kappa[IDX(g, ci, cj, kk)];
        }
        if (kbar > 0.0) {
            double G[4];
            orc_interp_gamma(g, r->x[i], r->y[i], r->z[i], G); /* K^2 includes Gamma^2 */
            K2 = (r->k[i] * r->k[i] + r->l[i] * r->l[i]) + (r->m[i] * r->m[i] + G[0]);
            fac = 1.0 - ((2.0 * kbar) * K2) * dt;
            if (fac < 0.0) fac = 0.0;
            r->n[i] = r->n[i] * fac;
        }
    }
    free(start);
    free(fill);
    free(order);
}

/* ------------------------------------------------------------------------
 * Full flux formulation (Section 2b, eq. fluxes:momentum, eq.
 * fluxes:temperature, eq. fluxes:buoyancy, eq. mean-flow-impact).
 * The momentum flux tensor, flux direction i (x, y, z) times momentum
 * component (u, v):
 *   rho <v_i u_j> = int [omega^2 cg_i kh_j N + f^2 (e_r x cg)_i (e_r x kh)_j N]
 *                   / (omega^2 - f^2) d^3k,
 * with e_r x a = (-a_y, a_x, 0), cg the intrinsic group velocity, and
 * omega^2 - f^2 = kh^2 (N^2 - f^2) / K^2 (no cancellation).  The potential-
 * temperature flux is deposited in its buoyancy form
 *   <u' b'> = (g / theta) <u' theta'> = int (1/rho) cg_z (f N^2 / (omega^2 - f^2))
 *             (e_r x kh) N d^3k,
 * which needs no reference potential temperature (a caller with theta
 * multiplies by theta / g).  Projection as the pseudo-momentum fluxes
 * (orc_deposit): the horizontal components are cell means over the carrier's
 * column, the vertical ones live on the staggered interfaces; rho of the
 * level, omega, cg, N^2, f and f^2 at the carrier.
 * Layout flux8 [8][nz+1][ny][nx]: Fxu, Fxv, Fyu, Fyv, Bu, Bv on levels
 * (slot nz = 0), Fzu, Fzv on interfaces.
 * ------------------------------------------------------------------------ */
static void full_flux_ray(const orc_bg *g, const orc_rays *r, int64_t i, int c, double *flux)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t colstride = (size_t)g->ny * (size_t)g->nx;
    int ci = c % g->nx, cj = c / g->nx;
    double B[14], D[4];
    double W = ray_W(r, i);
    double z = r->z[i], Dz = r->dz[i];
    double zb = z - 0.5 * Dz, zt = z + 0.5 * Dz;
    double Lz = (double)g->nz * g->dz;
    double k = r->k[i], l = r->l[i], m = r->m[i];
    double kh2 = k * k + l * l;
    double K2, G2;
    double N2, f2, fs, om2, den, a1, a2, v[8];
    int kk, klo, khi;
    corners cc;

    disp_at(g, r->x[i], r->y[i], z, k, l, m, B, D, &G2);
    K2 = kh2 + (m * m + G2);
    N2 = B[2];
    f2 = B[12];
    locate(g, r->x[i], r->y[i], z, &cc);
    fs = rowlin(g->f, &cc);
    om2 = D[0] * D[0];
    den = (kh2 * (N2 - f2)) / K2; /* omega^2 - f^2 */
    a1 = om2 / den;
    a2 = f2 / den;
    v[0] = a1 * (D[1] * k) + a2 * (D[2] * l); /* Fxu */
    v[1] = a1 * (D[1] * l) - a2 * (D[2] * k); /* Fxv */
    v[2] = a1 * (D[2] * k) - a2 * (D[1] * l); /* Fyu */
    v[3] = a1 * (D[2] * l) + a2 * (D[1] * k); /* Fyv */
    v[4] = -(((D[3] * fs) * N2) / den) * l;   /* Bu (times 1/rho at the level) */
    v[5] = (((D[3] * fs) * N2) / den) * k;    /* Bv */
    v[6] = a1 * (D[3] * k);                   /* Fzu */
    v[7] = a1 * (D[3] * l);                   /* Fzv */

    klo = (int)floor(zb / g->dz);
    khi = (int)floor(zt / g->dz);
    if (klo < 0) klo = 0;
    if (khi > g->nz - 1) khi = g->nz - 1;
    for (kk = klo; kk <= khi; kk++) {
        double lo = (double)kk * g->dz, hi = (double)(kk + 1) * g->dz;
        double o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        double frac, vol;
        size_t at;
        int q;
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, ((double)kk + 0.5) * g->dz) * g->dz;
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        for (q = 0; q < 4; q++) flux[(size_t)q * plane + at] += ((v[q] * W) * frac) / vol;
        for (q = 4; q < 6; q++) flux[(size_t)q * plane + at] += (((v[q] * W) * frac) / vol) / g->rho[kk];
    }
    klo = (int)floor(zb / g->dz + 0.5);
    khi = (int)floor(zt / g->dz + 0.5);
    if (klo < 0) klo = 0;
    if (khi > g->nz) khi = g->nz;
    for (kk = klo; kk <= khi; kk++) {
        double lo = ((double)kk - 0.5) * g->dz, hi = ((double)kk + 0.5) * g->dz;
        double o, frac, vol;
        size_t at;
        int q;
        if (lo < 0.0) lo = 0.0;
        if (hi > Lz) hi = Lz;
        o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, (double)kk * g->dz) * (hi - lo);
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        for (q = 6; q < 8; q++) flux[(size_t)q * plane + at] += ((v[q] * W) * frac) / vol;
    }
}

/* the active rays grouped by column in index order (a stable counting sort);
   with given_cols the keys already in r->col are used (see orc_saturation) */
static int64_t *column_order(const orc_bg *g, orc_rays *r, int64_t n, int given_cols, int64_t **start_out)
{
    int ncol = g->nx * g->ny;
    int64_t *start = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t i;
    int c;
    if (!given_cols) orc_keys(g, r, n);
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) start[r->col[i] + 1]++;
    for (c = 0; c < ncol; c++) start[c + 1] += start[c];
    for (i = 0; i < n; i++)
        if (r->state[i] == ORC_ACTIVE) {
            int cc = r->col[i];
            order[start[cc] + fill[cc]] = i;
            fill[cc]++;
        }
    free(fill);
    *start_out = start;
    return order;
}

void orc_full_fluxes(const orc_bg *g, orc_rays *r, int64_t n, double *flux8, int given_cols)
{
    int ncol = g->nx * g->ny;
    int64_t *start, *order = column_order(g, r, n, given_cols, &start);
    int c;
    memset(flux8, 0, (size_t)8 * (size_t)(g->nz + 1) * (size_t)ncol * sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (c = 0; c < ncol; c++) {
        int64_t p;
        for (p = start[c]; p < start[c + 1]; p++) full_flux_ray(g, r, order[p], c, flux8);
    }
    free(start);
    free(order);
}

/* ------------------------------------------------------------------------
 * Horizontal smoothing (Appendix B, horizontal flux smoothing): each cell
 * becomes the weighted mean of itself (weight 3), the cells sharing an edge
 * with it (weight 2) and the cells sharing only a corner (weight 1) -- the
 * ICON triangle weights carried over to the quadrilateral grid.  Periodic
 * in x (and y on the box); on the sphere the rows beyond the first and last
 * are left out and the weights of the present cells renormalised.  Applied
 * to nslices horizontal slices [nslices][ny][nx].
 * ------------------------------------------------------------------------ */
void orc_smooth(const orc_bg *g, const double *in, int nslices, double *out)
{
    size_t slice = (size_t)g->ny * (size_t)g->nx;
    int s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < nslices; s++) {
        const double *F = in + (size_t)s * slice;
        double *O = out + (size_t)s * slice;
        int i, j, di, dj;
        for (j = 0; j < g->ny; j++)
            for (i = 0; i < g->nx; i++) {
                double sum = 0.0, wsum = 0.0;
                for (dj = -1; dj <= 1; dj++) {
                    int jj = j + dj;
                    if (g->geometry == ORC_CARTESIAN) {
                        jj = (jj + g->ny) % g->ny;
                    } else if (jj < 0 || jj > g->ny - 1) {
                        continue;
                    }
                    for (di = -1; di <= 1; di++) {
                        int ii = (i + di + g->nx) % g->nx;
                        double w = (di == 0 && dj == 0) ? 3.0 : ((di == 0 || dj == 0) ? 2.0 : 1.0);
                        sum += w * F[(size_t)jj * (size_t)g->nx + (size_t)ii];
                        wsum += w;
                    }
                }
                O[(size_t)j * (size_t)g->nx + (size_t)i] = sum / wsum;
            }
    }
}

/* ------------------------------------------------------------------------
 * Divergence of a flux (Fx, Fy on levels [nz+1][ny][nx] with slot nz unused,
 * Fz on interfaces, Fz may be NULL) with the operator of orc_drag: centred
 * differences of the cell means (periodic; on the sphere (1/(r cos phi))
 * [d_lambda Fx + d_phi (cos phi Fy)], one-sided at the first and last rows)
 * plus the difference of the interface values across the level.
 * out [nz][ny][nx].
 * ------------------------------------------------------------------------ */
void orc_divergence(const orc_bg *g, const double *Fx, const double *Fy, const double *Fz, double *out)
{
    int i, j, k;
    for (k = 0; k < g->nz; k++)
        for (j = 0; j < g->ny; j++)
            for (i = 0; i < g->nx; i++) {
                int ip = (i + 1) % g->nx, im = (i + g->nx - 1) % g->nx;
                double divx, divy, divz;
                divz = Fz ? (Fz[IDX(g, i, j, k + 1)] - Fz[IDX(g, i, j, k)]) / g->dz : 0.0;
                if (g->geometry == ORC_CARTESIAN) {
                    int jp = (j + 1) % g->ny, jm = (j + g->ny - 1) % g->ny;
                    divx = (Fx[IDX(g, ip, j, k)] - Fx[IDX(g, im, j, k)]) / (2.0 * g->dx);
                    divy = (Fy[IDX(g, i, jp, k)] - Fy[IDX(g, i, jm, k)]) / (2.0 * g->dy);
                } else {
                    double r = g->a + ((double)k + 0.5) * g->dz;
                    double cj = cos(g->y0 + ((double)j + 0.5) * g->dy);
                    double rc = r * cj;
                    double dphi;
                    divx = ((Fx[IDX(g, ip, j, k)] - Fx[IDX(g, im, j, k)]) / (2.0 * g->dx)) / rc;
                    if (g->ny == 1) {
                        dphi = 0.0;
                    } else if (j == 0) {
                        double c1 = cos(g->y0 + 1.5 * g->dy);
                        dphi = (c1 * Fy[IDX(g, i, 1, k)] - cj * Fy[IDX(g, i, 0, k)]) / g->dy;
                    } else if (j == g->ny - 1) {
                        double cm = cos(g->y0 + ((double)j - 0.5) * g->dy);
                        dphi = (cj * Fy[IDX(g, i, j, k)] - cm * Fy[IDX(g, i, j - 1, k)]) / g->dy;
                    } else {
                        double cp = cos(g->y0 + ((double)j + 1.5) * g->dy);
                        double cm = cos(g->y0 + ((double)j - 0.5) * g->dy);
                        dphi = (cp * Fy[IDX(g, i, j + 1, k)] - cm * Fy[IDX(g, i, j - 1, k)]) / (2.0 * g->dy);
                    }
                    divy = dphi / rc;
                }
                out[IDX(g, i, j, k)] = (divx + divy) + divz;
            }
}

/* ------------------------------------------------------------------------
 * Mean-flow tendencies of the full formulation (eq. mean-flow-impact and
 * eq. mean-flow-impact-t in buoyancy form):
 *   du = -(1/rho) div(Fx u, Fy u, Fz u) - (f/g) Bv,
 *   dv = -(1/rho) div(Fx v, Fy v, Fz v) + (f/g) Bu,   ((f/g) e_r x <u'b'>)
 *   db = -div_h(Bu, Bv)   (the buoyancy tendency, (g/theta) dtheta/dt),
 * with f of the cell's row and g = 9.80665 m s^-2.  flux8 as written by
 * orc_full_fluxes (possibly smoothed); out3 [3][nz][ny][nx].
 * ------------------------------------------------------------------------ */
#define ORC_GRAVITY 9.80665
void orc_full_tendencies(const orc_bg *g, const double *flux8, double *out3)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t cells = (size_t)g->nz * (size_t)g->ny * (size_t)g->nx;
    double *div = (double *)malloc(sizeof(double) * cells);
    size_t at;
    int comp;
    for (comp = 0; comp < 2; comp++) {
        orc_divergence(g, flux8 + (size_t)comp * plane, flux8 + (size_t)(2 + comp) * plane,
                       flux8 + (size_t)(6 + comp) * plane, div);
        for (at = 0; at < cells; at++) {
            int k = (int)(at / ((size_t)g->ny * (size_t)g->nx));
            int j = (int)((at / (size_t)g->nx) % (size_t)g->ny);
            double fg = g->f[j] / ORC_GRAVITY;
            double el = comp == 0 ? -(fg * flux8[5 * plane + at]) : fg * flux8[4 * plane + at];
            out3[(size_t)comp * cells + at] = -(div[at] / g->rho[k]) + el;
        }
    }
    orc_divergence(g, flux8 + 4 * plane, flux8 + 5 * plane, NULL, div);
    for (at = 0; at < cells; at++) out3[2 * cells + at] = -div[at];
    free(div);
}

/* ------------------------------------------------------------------------
 * Wave-action budget fields (Section 4, eq. wave-action-budget): the wave
 * action per unit volume A = int N d^3k and its fluxes (cg_h A, cg_r A) =
 * int (cg_h, cg_r) N d^3k with the ground-based group velocity (U + cg_x,
 * V + cg_y, cg_z) at the carrier, projected like the fluxes.
 * fields4 [4][nz+1][ny][nx]: A, cgx A, cgy A on levels, cgz A on interfaces.
 * orc_budget_terms gives the horizontal and vertical propagation terms
 * div_h(cg_h A) and d_z(cg_z A), terms2 [2][nz][ny][nx].  The saturation term
 * is the change of A across orc_saturation divided by its time step.
 * ------------------------------------------------------------------------ */
static void budget_ray(const orc_bg *g, const orc_rays *r, int64_t i, int c, double *fields)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t colstride = (size_t)g->ny * (size_t)g->nx;
    int ci = c % g->nx, cj = c / g->nx;
    double B[14], D[4], v[4];
    double W = ray_W(r, i);
    double z = r->z[i], Dz = r->dz[i];
    double zb = z - 0.5 * Dz, zt = z + 0.5 * Dz;
    double Lz = (double)g->nz * g->dz;
    int kk, klo, khi;
    disp_at(g, r->x[i], r->y[i], z, r->k[i], r->l[i], r->m[i], B, D, NULL);
    v[0] = 1.0;
    v[1] = B[0] + D[1];
    v[2] = B[1] + D[2];
    v[3] = D[3];
    klo = (int)floor(zb / g->dz);
    khi = (int)floor(zt / g->dz);
    if (klo < 0) klo = 0;
    if (khi > g->nz - 1) khi = g->nz - 1;
    for (kk = klo; kk <= khi; kk++) {
        double lo = (double)kk * g->dz, hi = (double)(kk + 1) * g->dz;
        double o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        double frac, vol;
        size_t at;
        int q;
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, ((double)kk + 0.5) * g->dz) * g->dz;
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        for (q = 0; q < 3; q++) fields[(size_t)q * plane + at] += ((v[q] * W) * frac) / vol;
    }
    klo = (int)floor(zb / g->dz + 0.5);
    khi = (int)floor(zt / g->dz + 0.5);
    if (klo < 0) klo = 0;
    if (khi > g->nz) khi = g->nz;
    for (kk = klo; kk <= khi; kk++) {
        double lo = ((double)kk - 0.5) * g->dz, hi = ((double)kk + 0.5) * g->dz;
        double o, frac, vol;
        size_t at;
        if (lo < 0.0) lo = 0.0;
        if (hi > Lz) hi = Lz;
        o = (zt < hi ? zt : hi) - (zb > lo ? zb : lo);
        if (!(o > 0.0)) continue;
        frac = o / Dz;
        vol = cell_area(g, cj, (double)kk * g->dz) * (hi - lo);
        at = (size_t)kk * colstride + (size_t)cj * (size_t)g->nx + (size_t)ci;
        fields[3 * plane + at] += ((v[3] * W) * frac) / vol;
    }
}

void orc_budget(const orc_bg *g, orc_rays *r, int64_t n, double *fields4, int given_cols)
{
    int ncol = g->nx * g->ny;
    int64_t *start, *order = column_order(g, r, n, given_cols, &start);
    int c;
    memset(fields4, 0, (size_t)4 * (size_t)(g->nz + 1) * (size_t)ncol * sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (c = 0; c < ncol; c++) {
        int64_t p;
        for (p = start[c]; p < start[c + 1]; p++) budget_ray(g, r, order[p], c, fields4);
    }
    free(start);
    free(order);
}

void orc_budget_terms(const orc_bg *g, const double *fields4, double *terms2)
{
    size_t plane = (size_t)(g->nz + 1) * (size_t)g->ny * (size_t)g->nx;
    size_t cells = (size_t)g->nz * (size_t)g->ny * (size_t)g->nx;
    size_t at;
    int k, j, i;
    orc_divergence(g, fields4 + plane, fields4 + 2 * plane, NULL, terms2);
    for (k = 0; k < g->nz; k++)
        for (j = 0; j < g->ny; j++)
            for (i = 0; i < g->nx; i++) {
                at = IDX(g, i, j, k);
                terms2[cells + at] = (fields4[3 * plane + IDX(g, i, j, k + 1)] - fields4[3 * plane + at]) / g->dz;
            }
}

/* ------------------------------------------------------------------------
 * Continuous launch (Section 3c, sources): a ghost layer below the launch
 * height holds, in every column, the launch spectrum; each step the part of
 * it that has propagated up out of the layer during dt is separated and
 * activated as a new ray volume.
 *  - Column launch flux: flux_col[c] if given, else on the sphere the
 *    background source F_am(phi, t) = 1/2 [F_sol(phi)(1 + cos tau) +
 *    F_sol(-phi)(1 - cos tau)], tau = 2 pi t / year, F_sol(phi) = alpha(phi)
 *    F_s + alpha(-phi) F_w, phi of the row centre in degrees.
 *  - Spectrum: four horizontal directions (east, north, west, south) with a
 *    quarter of the flux each; intrinsic phase speeds c_b at the centres of
 *    n_speeds equal bins of [c_min, c_max], weighted by
 *    exp(-((c_b - c_center)/c_width)^2) normalised over the bins; one
 *    horizontal wavelength.
 *  - At the column centre at the launch height: omega_hat = kh c_b; a bin
 *    propagates vertically only for f^2 < omega_hat^2 < N^2 (the others are
 *    reflected in the ghost layer and discarded, their flux with them);
 *    m = -sqrt(kh^2 (N^2 - omega_hat^2) / (omega_hat^2 - f^2) - Gamma^2)
 *    (upward), from the dispersion relation with the scale-height
 *    correction; a bin for which the root is not positive is evanescent and
 *    discarded too.
 *  - New volume: what crossed the launch height during dt, from z_launch to
 *    z_launch + cg_z dt; horizontal extents one cell at the column centre;
 *    dk = dl = kh/10, dm = |m|/10; wave action W = F_bin A dt / kh (A the
 *    cell's area at the launch height), so that the volume carries the
 *    bin's pseudo-momentum flux; N = W / (Px Py Pz).
 * New volumes are appended in order of column, direction, phase speed, with
 * consecutive ids from *next_id.  Returns the new count, or -1 (nothing
 * changed) if the capacity is short.
 * ------------------------------------------------------------------------ */
#define ORC_PI 3.14159265358979323846
#define ORC_YEAR (365.25 * 86400.0)

static double source_alpha(double phi_deg)
{
    if (phi_deg >= 80.0) {
        double a = 1.0 - (phi_deg - 80.0) / 5.0;
        if (a < 0.0) a = 0.0;
        if (a > 1.0) a = 1.0;
        return a;
    }
    if (phi_deg >= 50.0) return 1.0;
    if (phi_deg >= 20.0) return 0.5 * (1.0 - cos(ORC_PI * (phi_deg - 20.0) / 30.0));
    return 0.0;
}

double orc_launch_flux(const orc_bg *g, int j, const orc_launch_params *p)
{
    double phi, tau, fsol_n, fsol_s;
    if (p->flux_col) return 0.0; /* per column: see orc_launch */
    if (g->geometry != ORC_SPHERICAL) return 0.0;
    phi = (g->y0 + ((double)j + 0.5) * g->dy) * (180.0 / ORC_PI);
    tau = (2.0 * ORC_PI) * (p->t_solstice / ORC_YEAR);
    fsol_n = source_alpha(phi) * p->F_s + source_alpha(-phi) * p->F_w;
    fsol_s = source_alpha(-phi) * p->F_s + source_alpha(phi) * p->F_w;
    return 0.5 * (fsol_n * (1.0 + cos(tau)) + fsol_s * (1.0 - cos(tau)));
}

int64_t orc_launch(const orc_bg *g, orc_rays *r, int64_t n, int64_t capacity, const orc_launch_params *p,
                   int64_t *next_id, orc_tally *t)
{
    static const double dir_k[4] = {1.0, 0.0, -1.0, 0.0};
    static const double dir_l[4] = {0.0, 1.0, 0.0, -1.0};
    int ncol = g->nx * g->ny;
    int pass, c, d, b;
    double sw = 0.0, kh = (2.0 * ORC_PI) / p->lambda_h;
    int64_t out = n, count = 0;
    for (b = 0; b < p->n_speeds; b++) {
        double cb = p->c_min + (((double)b + 0.5) * (p->c_max - p->c_min)) / (double)p->n_speeds;
        double s = (cb - p->c_center) / p->c_width;
        sw += exp(-(s * s));
    }
    for (pass = 0; pass < 2; pass++) {
        if (pass == 1 && n + count > capacity) return -1;
        for (c = 0; c < ncol; c++) {
            int i = c % g->nx, j = c / g->nx;
            double x = g->x0 + ((double)i + 0.5) * g->dx, y = g->y0 + ((double)j + 0.5) * g->dy;
            double Fc = p->flux_col ? p->flux_col[c] : orc_launch_flux(g, j, p);
            double B[14], G[4];
            if (!(Fc > 0.0)) continue;
            orc_interp(g, x, y, p->z_launch, B);
            orc_interp_gamma(g, x, y, p->z_launch, G);
            for (d = 0; d < 4; d++)
                for (b = 0; b < p->n_speeds; b++) {
                    double cb = p->c_min + (((double)b + 0.5) * (p->c_max - p->c_min)) / (double)p->n_speeds;
                    double s = (cb - p->c_center) / p->c_width;
                    double Fb = (0.25 * Fc) * (exp(-(s * s)) / sw);
                    double om = kh * cb, om2 = om * om, N2 = B[2], f2 = B[12];
                    double m, m2, k, l, D[4], Dz, z, A, W, dk, dm, px, py, pz;
                    int64_t o;
                    if (!(om2 > f2 && om2 < N2) || !(Fb > 0.0)) continue;
                    m2 = ((kh * kh) * (N2 - om2)) / (om2 - f2) - G[0];
                    if (!(m2 > 0.0)) continue; /* evanescent: Gamma^2 exceeds m^2 + Gamma^2 */
                    if (pass == 0) {
                        count++;
                        continue;
                    }
                    m = -sqrt(m2);
                    k = kh * dir_k[d];
                    l = kh * dir_l[d];
                    orc_dispersion_g(N2, f2, G[0], k, l, m, D);
                    Dz = D[3] * p->dt;
                    z = p->z_launch + 0.5 * Dz;
                    A = cell_area(g, j, p->z_launch);
                    W = ((Fb * A) * p->dt) / kh;
                    dk = 0.1 * kh;
                    dm = 0.1 * fabs(m);
                    px = metric_x(g, y, z, g->dx) * dk;
                    py = metric_y(g, z, g->dy) * dk;
                    pz = Dz * dm;
                    o = out++;
                    r->x[o] = x;
                    r->y[o] = y;
                    r->z[o] = z;
                    r->k[o] = k;
                    r->l[o] = l;
                    r->m[o] = m;
                    r->dx[o] = g->dx;
                    r->dy[o] = g->dy;
                    r->dz[o] = Dz;
                    r->px[o] = px;
                    r->py[o] = py;
                    r->pz[o] = pz;
                    r->n[o] = W / ((px * py) * pz);
                    r->id[o] = (*next_id)++;
                    r->state[o] = ORC_ACTIVE;
                    r->col[o] = c;
                    if (t) {
                        t->n_launched++;
                        t->launched_W += W;
                    }
                }
        }
    }
    return out;
}
