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
// arithmetic: a context has fewer than 2^24 columns)
__global__ __launch_bounds__(256) void k_drag(Grid g, const double *__restrict__ rho, const double *__restrict__ cosr,
                                              const double *__restrict__ flux, double *__restrict__ drag)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    const uint32_t col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= (uint32_t)g.ncol) return;
    const int k = (int)blockIdx.y;
    const int j = (int)(col / (uint32_t)g.nx);
    const int i = (int)col - j * g.nx;
    const int64_t c = (int64_t)k * g.ncol + col;
    const int64_t plane = (int64_t)(g.nz + 1) * g.ncol;
    const int64_t row = g.nx;
    const int64_t at = (int64_t)k * g.ncol + (int64_t)j * g.nx + i;
    const int ip = i + 1 == g.nx ? 0 : i + 1, im = i == 0 ? g.nx - 1 : i - 1;
    for (int comp = 0; comp < 2; comp++) {
        const double *Fx = flux + (int64_t)(0 + comp) * plane;
        const double *Fy = flux + (int64_t)(2 + comp) * plane;
        const double *Fz = flux + (int64_t)(4 + comp) * plane;
        const double divz = (Fz[at + g.ncol] - Fz[at]) / g.dz;
        double divx, divy;
        if (g.geometry == RT_CARTESIAN) {
            const int jp = j + 1 == g.ny ? 0 : j + 1, jm = j == 0 ? g.ny - 1 : j - 1;
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
                const double c1 = cosr[1];
                dphi = (c1 * Fy[at + row] - cj * Fy[at]) / g.dy;
            } else if (j == g.ny - 1) {
                const double cm = cosr[j - 1];
                dphi = (cj * Fy[at] - cm * Fy[at - row]) / g.dy;
            } else {
                const double cp = cosr[j + 1];
                const double cm = cosr[j - 1];
                dphi = (cp * Fy[at + row] - cm * Fy[at - row]) / (2.0 * g.dy);
            }
            divy = dphi / rc;
        }
        drag[(int64_t)comp * cells + c] = -((divx + divy) + divz) / rho[k];
    }
}

void launch_drag(const Grid &g, const double *rho, const double *cosr, const double *flux, double *drag, hipStream_t s)
{
    if (g.nz <= 0 || g.ncol <= 0) return;
    k_drag<<<dim3((unsigned)((g.ncol + 255) / 256), (unsigned)g.nz), 256, 0, s>>>(g, rho, cosr, flux, drag);
}
