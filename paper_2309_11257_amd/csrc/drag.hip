// Wave drag from the deposited fluxes (eq. mean-flow-impact with the
// pseudo-momentum flux of Appendix A): du = -(1/rho) div(Fk), dv likewise with
// Fl.  Horizontal divergence by centred differences of the cell-mean fluxes
// (periodic; on the sphere (1/(r cos phi)) [d_lambda Fx + d_phi(cos phi Fy)]
// with one-sided differences at the first and last rows), vertical
// divergence as the difference of the interface fluxes across the level.
// One thread per cell; HBM-bound stencil.  The cosines of the row-centre
// latitudes come from a per-row table (the same cos() of the same argument,
// computed once).  Built with -ffp-contract=off.
#include "rt_internal.h"

__global__ void k_coslat(Grid g, double *cosr)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < g.ny) cosr[j] = cos(g.y0 + ((double)j + 0.5) * g.dy);
}

void launch_coslat(const Grid &g, double *cosr, hipStream_t s)
{
    k_coslat<<<(unsigned)((g.ny + 255) / 256), 256, 0, s>>>(g, cosr);
}

// grid: x over the columns of a level, y over the levels (32-bit column
// arithmetic: a context has fewer than 2^24 columns).  The grid spacings'
// reciprocals come from the host, and each thread forms 1/rho and 1/(r cos
// phi) once for both components: products instead of twelve correctly
// rounded divisions per cell (a few units in the last place from the
// oracle's quotients, far below the deposition's own rounding).
struct DragInv {
    double dz, dx2, dy2, dy;  // 1/dz, 1/(2 dx), 1/(2 dy), 1/dy
};

__global__ __launch_bounds__(256) void k_drag(Grid g, DragInv inv, const double *__restrict__ rho,
                                              const double *__restrict__ cosr, const double *__restrict__ flux,
                                              double *__restrict__ drag)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    // runs of consecutive blocks of a level stay on one XCD (the flux rows of
    // neighbouring columns share its L2)
    const int64_t lb = xcd_lin((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
    const uint32_t col = (uint32_t)(lb % gridDim.x) * blockDim.x + threadIdx.x;
    if (col >= (uint32_t)g.ncol) return;
    const int k = (int)(lb / gridDim.x);
    const int j = (int)(col / (uint32_t)g.nx);
    const int i = (int)col - j * g.nx;
    const int64_t c = (int64_t)k * g.ncol + col;
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const int64_t row = g.nx;
    const int64_t at = (int64_t)k * g.ncol + (int64_t)j * g.nx + i;
    const int ip = i + 1 == g.nx ? 0 : i + 1, im = i == 0 ? g.nx - 1 : i - 1;
    const double irho = 1.0 / rho[k];
    const bool sph = g.geometry != RT_CARTESIAN;
    double irc = 1.0, cj = 1.0, cp = 1.0, cm = 1.0;
    if (sph) {
        const double r = g.a + ((double)k + 0.5) * g.dz;
        cj = cosr[j];
        irc = 1.0 / (r * cj);
        cp = j + 1 < g.ny ? cosr[j + 1] : 0.0;
        cm = j > 0 ? cosr[j - 1] : 0.0;
    }
    for (int comp = 0; comp < 2; comp++) {
        const double *Fx = flux + (int64_t)(0 + comp) * plane;
        const double *Fy = flux + (int64_t)(2 + comp) * plane;
        const double *Fz = flux + (int64_t)(4 + comp) * plane;
        const double divz = (Fz[at + g.ncol] - Fz[at]) * inv.dz;
        const double dlam = (Fx[at - i + ip] - Fx[at - i + im]) * inv.dx2;
        double hdiv;
        if (!sph) {
            const int jp = j + 1 == g.ny ? 0 : j + 1, jm = j == 0 ? g.ny - 1 : j - 1;
            hdiv = dlam + (Fy[at + (jp - j) * row] - Fy[at + (jm - j) * row]) * inv.dy2;
        } else {
            double dphi;
            if (g.ny == 1)
                dphi = 0.0;
            else if (j == 0)
                dphi = (cp * Fy[at + row] - cj * Fy[at]) * inv.dy;
            else if (j == g.ny - 1)
                dphi = (cj * Fy[at] - cm * Fy[at - row]) * inv.dy;
            else
                dphi = (cp * Fy[at + row] - cm * Fy[at - row]) * inv.dy2;
            hdiv = (dlam + dphi) * irc;
        }
        drag[(int64_t)comp * cells + c] = -(hdiv + divz) * irho;
    }
}

void launch_drag(const Grid &g, const double *rho, const double *cosr, const double *flux, double *drag, hipStream_t s)
{
    if (g.nz <= 0 || g.ncol <= 0) return;
    const DragInv inv{1.0 / g.dz, 1.0 / (2.0 * g.dx), 1.0 / (2.0 * g.dy), 1.0 / g.dy};
    k_drag<<<dim3((unsigned)((g.ncol + 255) / 256), (unsigned)g.nz), 256, 0, s>>>(g, inv, rho, cosr, flux, drag);
}
