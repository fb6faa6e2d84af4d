// Full flux formulation, horizontal smoothing and wave-action budget.
//
// Full fluxes (Section 2b, eq. fluxes:momentum, eq. fluxes:temperature, eq.
// fluxes:buoyancy): per volume the momentum flux tensor
//   [omega^2 cg_i kh_j + f^2 (e_r x cg)_i (e_r x kh)_j] / (omega^2 - f^2) W
// (e_r x a = (-a_y, a_x, 0); omega^2 - f^2 = kh^2 (N^2 - f^2) / K^2, free of
// cancellation) and the buoyancy flux cg_z f N^2 / (omega^2 - f^2) (e_r x kh) W,
// deposited with the per-column machinery as eight fields: Fxu, Fxv, Fyu,
// Fyv, Bu, Bv on levels, Fzu, Fzv on interfaces; Bu, Bv are then divided by
// the level's reference density.  The tendencies are
//   du = -(1/rho) div(Fxu, Fyu, Fzu) - (f/g) Bv,   dv = -(1/rho) div(Fxv, Fyv, Fzv) + (f/g) Bu,
//   db = -div_h(Bu, Bv)
// (eq. mean-flow-impact: the elastic term (f/g) e_r x <u'b'>; eq.
// mean-flow-impact-t in buoyancy form).
// Budget (Section 4, eq. wave-action-budget): A, (U + cg_x) A, (V + cg_y) A on
// levels and cg_z A on interfaces, and their propagation terms.
// Smoothing (Appendix B): weights 3 (centre), 2 (edge neighbours), 1 (corner
// neighbours), periodic in x (and y on the box), the sphere's missing rows
// left out with the weights renormalised.
// Built with -ffp-contract=off: the double-precision path evaluates every
// expression in the order the definitions are written.
#include "dev64.h"
#include "f32.h"
#include "deposit_common.h"

#define GRAVITY 9.80665

struct PayFull64 {
    Grid g;
    Bg64P b;
    S64 st;
    const double *frow;  // signed Coriolis parameter by latitude row
    double inv_dz;       // unused: the double-precision levels divide
    static constexpr bool EXACT_LEVELS = true;
    static constexpr int NL = 6, NI = 2;
    static constexpr int WAVES = 4;  // eight or four fields and more live values
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        (void)col;
        const double x = st.x[s], y = st.y[s], z = st.z[s];
        const double k = st.k[s], l = st.l[s], m = st.m[s], Dz = st.dz[s];
        const double W = st.W[s];
        const d64::Axis ay = d64::axis_y(g, y);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, x), ay, d64::axis_z(g, z));
        const d64::Corners<1> K(b.A, c, 0);
        const double N2 = TRI64(K, z, c);
        const double f2 = d64::row_lerp(b.f2, ay);
        const double fs = d64::row_lerp(frow, ay);
        const double kh2 = k * k + l * l;
        const double M2 = m * m + d64::gam2(b, c);
        const double K2 = kh2 + M2;
        const double K4 = K2 * K2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        const double d = N2 - f2;
        const double dn = om * K4;
        const double cx = ((k * M2) * d) / dn;
        const double cy = ((l * M2) * d) / dn;
        const double cz = -(((m * kh2) * d) / dn);
        const double om2 = om * om;
        const double den = (kh2 * (N2 - f2)) / K2;
        const double a1 = om2 / den, a2 = f2 / den;
        const double bf = ((cz * fs) * N2) / den;
        const double sW = W / Dz;
        bv[0] = (a1 * (cx * k) + a2 * (cy * l)) * sW;
        bv[1] = (a1 * (cx * l) - a2 * (cy * k)) * sW;
        bv[2] = (a1 * (cy * k) - a2 * (cx * l)) * sW;
        bv[3] = (a1 * (cy * l) + a2 * (cx * k)) * sW;
        bv[4] = (-bf * l) * sW;
        bv[5] = (bf * k) * sW;
        bv[6] = (a1 * (cz * k)) * sW;
        bv[7] = (a1 * (cz * l)) * sW;
        zb = z - 0.5 * Dz;
        zt = z + 0.5 * Dz;
    }
};

struct PayFull32 {
    G32 g;
    Bg32P b;
    S32 st;
    const float *frow;
    double zdz, inv_dz;
    static constexpr bool EXACT_LEVELS = false;
    static constexpr int NL = 6, NI = 2;
    static constexpr int WAVES = 4;  // eight or four fields and more live values
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        const int jc = (int)((uint32_t)col / (uint32_t)g.nx), ic = col - jc * g.nx;
        const int kc = st.lev[s];
        const float zeta = st.zeta[s], eta = st.eta[s];
        const float k = st.k[s], l = st.l[s], m = (float)st.m[s];
        const float Dz = st.dz[s];
        float N2, f2;
        f32::n2_f2(g, b, ic, jc, kc, st.xi[s], eta, zeta, N2, f2);
        const float fs = f32::row_lerp(frow, f32::axis_y(g, jc, eta));
        const float kh2 = k * k + l * l;
        const float M2 = m * m + f32::gam2_at(g, b, ic, jc, kc, st.xi[s], eta, zeta);
        const float K2 = kh2 + M2;
        const float invK2 = f32::rcp(K2);
        const float rom = f32::rsq((N2 * kh2 + f2 * M2) * invK2);  // 1 / omega_hat
        const float sc = (N2 - f2) * (invK2 * invK2) * rom;
        const float cx = k * M2 * sc, cy = l * M2 * sc, cz = -m * kh2 * sc;
        const float om2 = (N2 * kh2 + f2 * M2) * invK2;
        const float iden = K2 * f32::rcp(kh2 * (N2 - f2));  // 1 / (omega^2 - f^2)
        const float a1 = om2 * iden, a2 = f2 * iden;
        const float bf = cz * fs * N2 * iden;
        const double sW = st.W[s] * (double)f32::rcp(Dz);
        bv[0] = (double)(a1 * cx * k + a2 * cy * l) * sW;
        bv[1] = (double)(a1 * cx * l - a2 * cy * k) * sW;
        bv[2] = (double)(a1 * cy * k - a2 * cx * l) * sW;
        bv[3] = (double)(a1 * cy * l + a2 * cx * k) * sW;
        bv[4] = (double)(-bf * l) * sW;
        bv[5] = (double)(bf * k) * sW;
        bv[6] = (double)(a1 * cz * k) * sW;
        bv[7] = (double)(a1 * cz * l) * sW;
        const double zc = ((double)kc + (double)zeta) * zdz;
        zb = zc - 0.5 * (double)Dz;
        zt = zc + 0.5 * (double)Dz;
    }
};

struct PayBudget64 {
    Grid g;
    Bg64P b;
    S64 st;
    double inv_dz;
    static constexpr bool EXACT_LEVELS = true;
    static constexpr int NL = 3, NI = 1;
    static constexpr int WAVES = 4;  // eight or four fields and more live values
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        (void)col;
        const double x = st.x[s], y = st.y[s], z = st.z[s];
        const double k = st.k[s], l = st.l[s], m = st.m[s], Dz = st.dz[s];
        const double W = st.W[s];
        const d64::Axis ay = d64::axis_y(g, y);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, x), ay, d64::axis_z(g, z));
        const d64::Corners<1> K(b.A, c, 0);
        const double U = TRI64(K, x, c), V = TRI64(K, y, c), N2 = TRI64(K, z, c);
        const double f2 = d64::row_lerp(b.f2, ay);
        const double kh2 = k * k + l * l;
        const double M2 = m * m + d64::gam2(b, c);
        const double K2 = kh2 + M2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        const double d = N2 - f2;
        const double dn = om * (K2 * K2);
        const double sW = W / Dz;
        bv[0] = 1.0 * sW;
        bv[1] = (U + ((k * M2) * d) / dn) * sW;
        bv[2] = (V + ((l * M2) * d) / dn) * sW;
        bv[3] = (-(((m * kh2) * d) / dn)) * sW;
        zb = z - 0.5 * Dz;
        zt = z + 0.5 * Dz;
    }
};

struct PayBudget32 {
    G32 g;
    Bg32P b;
    S32 st;
    double zdz, inv_dz;
    static constexpr bool EXACT_LEVELS = false;
    static constexpr int NL = 3, NI = 1;
    static constexpr int WAVES = 6;
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        const int jc = (int)((uint32_t)col / (uint32_t)g.nx), ic = col - jc * g.nx;
        const int kc = st.lev[s];
        const float zeta = st.zeta[s];
        const float k = st.k[s], l = st.l[s], m = (float)st.m[s];
        const float Dz = st.dz[s];
        const f32::Axis ax = f32::axis_per(ic, st.xi[s], g.nx), ay = f32::axis_y(g, jc, st.eta[s]);
        const f32::Cell c = f32::cell_of(g, ax, ay, f32::axis_clamp(kc, zeta, g.nz));
        const f32::Corners<1> K(b.A, c, 0);
        const float U = TRI_COMP(K, x, c), V = TRI_COMP(K, y, c), N2 = TRI_COMP(K, z, c);
        const float f2 = f32::row_lerp(b.f2, ay);
        const float kh2 = k * k + l * l;
        const float M2 = m * m + f32::gam2(b, c);
        const float invK2 = f32::rcp(kh2 + M2);
        const float rom = f32::rsq((N2 * kh2 + f2 * M2) * invK2);
        const float sc = (N2 - f2) * (invK2 * invK2) * rom;
        const double sW = st.W[s] * (double)f32::rcp(Dz);
        bv[0] = sW;
        bv[1] = (double)(U + k * M2 * sc) * sW;
        bv[2] = (double)(V + l * M2 * sc) * sW;
        bv[3] = (double)(-m * kh2 * sc) * sW;
        const double zc = ((double)kc + (double)zeta) * zdz;
        zb = zc - 0.5 * (double)Dz;
        zt = zc + 0.5 * (double)Dz;
    }
};

// Bu, Bv of the full fluxes divided by the level's reference density
__global__ void k_div_rho(Grid g, double *__restrict__ B, const double *__restrict__ rho)
{
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const int64_t at = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (at >= 2 * plane) return;
    const int kk = (int)((at % plane) / g.ncol);
    if (kk < g.nz) B[at] = B[at] / rho[kk];
}

// 3/2/1-weighted horizontal smoothing of nslices [ny][nx] slices
__global__ void k_smooth(Grid g, const double *__restrict__ in, double *__restrict__ out, int64_t nslices)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nslices * g.ncol) return;
    const int64_t s = e / g.ncol;
    const int c = (int)(e % g.ncol);
    const int i = c % g.nx, j = c / g.nx;
    const double *F = in + s * g.ncol;
    double sum = 0.0, wsum = 0.0;
    for (int dj = -1; dj <= 1; dj++) {
        int jj = j + dj;
        if (g.geometry == RT_CARTESIAN)
            jj = (jj + g.ny) % g.ny;
        else if (jj < 0 || jj > g.ny - 1)
            continue;
        for (int di = -1; di <= 1; di++) {
            const int ii = (i + di + g.nx) % g.nx;
            const double w = (di == 0 && dj == 0) ? 3.0 : ((di == 0 || dj == 0) ? 2.0 : 1.0);
            sum += w * F[(int64_t)jj * g.nx + ii];
            wsum += w;
        }
    }
    out[e] = sum / wsum;
}

// divergence of (Fx, Fy) on levels plus the interface difference of Fz (may
// be null) at cell (i, j, k): the operator of the drag
__device__ inline double div_at(const Grid &g, const double *__restrict__ cosr, const double *__restrict__ Fx,
                                const double *__restrict__ Fy, const double *__restrict__ Fz, int i, int j, int k)
{
    const int64_t row = g.nx;
    const int64_t at = (int64_t)k * g.ncol + (int64_t)j * g.nx + i;
    const int ip = (i + 1) % g.nx, im = (i + g.nx - 1) % g.nx;
    const double divz = Fz ? (Fz[at + g.ncol] - Fz[at]) / g.dz : 0.0;
    double divx, divy;
    if (g.geometry == RT_CARTESIAN) {
        const int jp = (j + 1) % g.ny, jm = (j + g.ny - 1) % g.ny;
        divx = (Fx[at - i + ip] - Fx[at - i + im]) / (2.0 * g.dx);
        divy = (Fy[at + (jp - j) * row] - Fy[at + (jm - j) * row]) / (2.0 * g.dy);
    } else {
        const double r = g.a + ((double)k + 0.5) * g.dz;
        const double cj = cosr[j];
        const double rc = r * cj;
        double dphi;
        divx = ((Fx[at - i + ip] - Fx[at - i + im]) / (2.0 * g.dx)) / rc;
        if (g.ny == 1) {
            dphi = 0.0;
        } else if (j == 0) {
            dphi = (cosr[1] * Fy[at + row] - cj * Fy[at]) / g.dy;
        } else if (j == g.ny - 1) {
            dphi = (cj * Fy[at] - cosr[j - 1] * Fy[at - row]) / g.dy;
        } else {
            dphi = (cosr[j + 1] * Fy[at + row] - cosr[j - 1] * Fy[at - row]) / (2.0 * g.dy);
        }
        divy = dphi / rc;
    }
    return (divx + divy) + divz;
}

// du, dv, db [3][nz][ny][nx] from the eight full-flux fields
__global__ void k_full_tend(Grid g, const double *__restrict__ cosr, const double *__restrict__ rho,
                            const double *__restrict__ frow, const double *__restrict__ F, double *__restrict__ out)
{
    const int64_t cells = (int64_t)g.nz * g.ncol;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / g.ncol);
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const int64_t at = (int64_t)k * g.ncol + (int64_t)j * g.nx + i;
    const double fg = frow[j] / GRAVITY;
    const double du = div_at(g, cosr, F, F + 2 * plane, F + 6 * plane, i, j, k);
    const double dv = div_at(g, cosr, F + plane, F + 3 * plane, F + 7 * plane, i, j, k);
    const double db = div_at(g, cosr, F + 4 * plane, F + 5 * plane, nullptr, i, j, k);
    out[c] = -(du / rho[k]) + -(fg * F[5 * plane + at]);
    out[cells + c] = -(dv / rho[k]) + fg * F[4 * plane + at];
    out[2 * cells + c] = -db;
}

// horizontal and vertical propagation terms [2][nz][ny][nx] of the budget
__global__ void k_budget_terms(Grid g, const double *__restrict__ cosr, const double *__restrict__ F,
                               double *__restrict__ out)
{
    const int64_t cells = (int64_t)g.nz * g.ncol;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / g.ncol);
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const int64_t at = (int64_t)k * g.ncol + (int64_t)j * g.nx + i;
    out[c] = div_at(g, cosr, F + plane, F + 2 * plane, nullptr, i, j, k);
    out[cells + c] = (F[3 * plane + at + g.ncol] - F[3 * plane + at]) / g.dz;
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_full_fluxes64(const Grid &g, const Bg64P &b, S64 st, const double *frow, const uint32_t *perm,
                          const uint32_t *colstart, const double *rho, double *F, hipStream_t s)
{
    PayFull64 p{g, b, st, frow, 1.0 / g.dz};
    launch_deposit_k(g, p, perm, colstart, F, s);
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    k_div_rho<<<nblk(2 * plane), 256, 0, s>>>(g, F + 4 * plane, rho);
}

void launch_full_fluxes32(const Grid &g, const Bg32P &b, S32 st, const float *frow, const uint32_t *perm,
                          const uint32_t *colstart, const double *rho, double *F, hipStream_t s)
{
    PayFull32 p{f32::make_g32(g), b, st, frow, g.dz, 1.0 / g.dz};
    launch_deposit_k(g, p, perm, colstart, F, s);
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    k_div_rho<<<nblk(2 * plane), 256, 0, s>>>(g, F + 4 * plane, rho);
}

void launch_budget64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart, double *F,
                     hipStream_t s)
{
    PayBudget64 p{g, b, st, 1.0 / g.dz};
    launch_deposit_k(g, p, perm, colstart, F, s);
}

void launch_budget32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart, double *F,
                     hipStream_t s)
{
    PayBudget32 p{f32::make_g32(g), b, st, g.dz, 1.0 / g.dz};
    launch_deposit_k(g, p, perm, colstart, F, s);
}

void launch_smooth(const Grid &g, const double *in, double *out, int64_t nslices, hipStream_t s)
{
    if (nslices > 0) k_smooth<<<nblk(nslices * g.ncol), 256, 0, s>>>(g, in, out, nslices);
}

void launch_full_tend(const Grid &g, const double *cosr, const double *rho, const double *frow, const double *F,
                      double *out, hipStream_t s)
{
    k_full_tend<<<nblk((int64_t)g.nz * g.ncol), 256, 0, s>>>(g, cosr, rho, frow, F, out);
}

void launch_budget_terms(const Grid &g, const double *cosr, const double *F, double *out, hipStream_t s)
{
    k_budget_terms<<<nblk((int64_t)g.nz * g.ncol), 256, 0, s>>>(g, cosr, F, out);
}
