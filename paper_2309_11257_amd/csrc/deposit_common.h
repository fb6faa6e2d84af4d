// Per-column flux deposition shared by both precisions.
//
// Ray volumes arrive grouped by column (radix sort on the column key).  One
// 256-thread workgroup owns DEP_CPW consecutive columns and, column after
// column, walks each column's volumes in chunks of 256 in sorted order; the
// finished profiles are written together so that the DEP_CPW columns of one
// (field, level) row form one 32-byte segment of the [6][nz+1][ncol] output.  Within a chunk every contribution is converted to an
// integer in a fixed-point format chosen from the chunk's largest
// contribution (2^51 units for that value) and added into an int64 profile in
// LDS; integer addition is associative, so the chunk total does not depend on
// the order in which lanes arrive.  Chunk totals are added to a double
// profile in chunk order.  The result is therefore bitwise reproducible from
// run to run, with no floating-point atomics, and each contribution is
// rounded once at the level of the chunk maximum's last bit -- the accuracy of
// an ordinary double sum.
#pragma once
#include "rt_internal.h"

// P::load(slot, zb, zt, bv[6]) fills the vertical span of the volume and its
// six flux densities per unit height: (cgx k, cgx l, cgy k, cgy l, cgz k,
// cgz l) * W / Dz.
#define DEP_CPW 4

// round x * scale (scale a power of two, |x * scale| <= 2^51) to the nearest
// integer, ties to even: adding 1.5 * 2^52 puts the integer part in the low
// mantissa bits of a double whose unit in the last place is 1
__device__ inline long long to_fixed(double x, double scale)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = x * scale + magic;
    return (long long)(__double_as_longlong(y) - __double_as_longlong(magic));
}

template <class P>
__global__ __launch_bounds__(256) void k_deposit(Grid g, P pl, const uint32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ colstart, double *__restrict__ flux)
{
    extern __shared__ unsigned long long dep_smem[];
    const int nzp = g.nz + 1;
    unsigned long long *acc = dep_smem;                   // [6][nzp]
    double *profs = (double *)(dep_smem + 6 * nzp);       // [DEP_CPW][6][nzp]
    __shared__ double wmax[4][6];
    __shared__ int sexp[6];
    const int c_first = blockIdx.x * DEP_CPW;
    const int ncols = min(DEP_CPW, g.ncol - c_first);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < 6 * nzp; e += 256) acc[e] = 0ull;
    for (int e = tid; e < DEP_CPW * 6 * nzp; e += 256) profs[e] = 0.0;
    __syncthreads();
    for (int cl = 0; cl < ncols; cl++) {
        const int c = c_first + cl;
        double *prof = profs + (size_t)cl * 6 * nzp;
        const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
        for (uint32_t base = s0; base < s1; base += 256) {
            const uint32_t r = base + (uint32_t)tid;
            const bool valid = r < s1;
            double zb = 0.0, zt = 0.0, bv[6] = {0, 0, 0, 0, 0, 0};
            if (valid) pl.load(perm[r], zb, zt, bv);
            const double h = valid ? fmin(zt - zb, g.dz) : 0.0;
            double mv[6];
    #pragma unroll
            for (int q = 0; q < 6; q++) mv[q] = fabs(bv[q]) * h;
    #pragma unroll
            for (int q = 0; q < 6; q++)
                for (int off = 32; off > 0; off >>= 1) mv[q] = fmax(mv[q], __shfl_xor(mv[q], off, 64));
            if (lane == 0)
    #pragma unroll
                for (int q = 0; q < 6; q++) wmax[wave][q] = mv[q];
            __syncthreads();
            if (tid < 6) {
                double m = fmax(fmax(wmax[0][tid], wmax[1][tid]), fmax(wmax[2][tid], wmax[3][tid]));
                int e = 0;
                if (m > 0.0 && m < 1.0e300) {
                    frexp(m, &e);
                    sexp[tid] = 51 - e;
                } else {
                    sexp[tid] = 0;
                }
            }
            __syncthreads();
            if (valid) {
                double sc[6];
    #pragma unroll
                for (int q = 0; q < 6; q++) sc[q] = ldexp(1.0, sexp[q]);
                int klo = (int)floor(zb / g.dz), khi = (int)floor(zt / g.dz);
                if (klo < 0) klo = 0;
                if (khi > g.nz - 1) khi = g.nz - 1;
                for (int kk = klo; kk <= khi; kk++) {
                    const double lo = (double)kk * g.dz, hi = (double)(kk + 1) * g.dz;
                    const double o = fmin(zt, hi) - fmax(zb, lo);
                    if (!(o > 0.0)) continue;
    #pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const long long v = to_fixed(bv[q] * o, sc[q]);
                        if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                    }
                }
                klo = (int)floor(zb / g.dz + 0.5);
                khi = (int)floor(zt / g.dz + 0.5);
                if (klo < 0) klo = 0;
                if (khi > g.nz) khi = g.nz;
                for (int kk = klo; kk <= khi; kk++) {
                    double lo = ((double)kk - 0.5) * g.dz, hi = ((double)kk + 0.5) * g.dz;
                    if (lo < 0.0) lo = 0.0;
                    if (hi > g.Lz) hi = g.Lz;
                    const double o = fmin(zt, hi) - fmax(zb, lo);
                    if (!(o > 0.0)) continue;
    #pragma unroll
                    for (int q = 4; q < 6; q++) {
                        const long long v = to_fixed(bv[q] * o, sc[q]);
                        if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                    }
                }
            }
            __syncthreads();
            for (int e = tid; e < 6 * nzp; e += 256) {
                const long long v = (long long)acc[e];
                if (v) {
                    prof[e] += ldexp((double)v, -sexp[e / nzp]);
                    acc[e] = 0ull;
                }
            }
            __syncthreads();
        }
    }  // columns of this workgroup
    // divide by the cell volume (levels) or staggered-cell volume (interfaces);
    // consecutive threads take consecutive columns of one (field, level) row
    for (int e = tid; e < DEP_CPW * 6 * nzp; e += 256) {
        const int cl = e % DEP_CPW, qk = e / DEP_CPW;
        const int q = qk / nzp, kk = qk % nzp;
        if (cl >= ncols) continue;
        const int c = c_first + cl;
        const int cj = c / g.nx;
        double area_h = g.dx * g.dy, cphi = 1.0;
        if (g.geometry == RT_SPHERICAL) cphi = cos(g.y0 + ((double)cj + 0.5) * g.dy);
        const double acc_v = profs[(size_t)cl * 6 * nzp + qk];
        double val;
        if (q < 4) {
            if (kk == g.nz) {
                val = 0.0;
            } else {
                double area = area_h;
                if (g.geometry == RT_SPHERICAL) {
                    const double rr = g.a + ((double)kk + 0.5) * g.dz;
                    area = (((rr * rr) * cphi) * g.dx) * g.dy;
                }
                val = acc_v / (area * g.dz);
            }
        } else {
            double lo = ((double)kk - 0.5) * g.dz, hi = ((double)kk + 0.5) * g.dz;
            if (lo < 0.0) lo = 0.0;
            if (hi > g.Lz) hi = g.Lz;
            double area = area_h;
            if (g.geometry == RT_SPHERICAL) {
                const double rr = g.a + (double)kk * g.dz;
                area = (((rr * rr) * cphi) * g.dx) * g.dy;
            }
            val = acc_v / (area * (hi - lo));
        }
        flux[((size_t)q * nzp + kk) * (size_t)g.ncol + c] = val;
    }
}

inline size_t deposit_smem(const Grid &g) { return (size_t)(6 + 6 * DEP_CPW) * (size_t)(g.nz + 1) * 8; }
inline unsigned deposit_blocks(const Grid &g) { return (unsigned)((g.ncol + DEP_CPW - 1) / DEP_CPW); }
