// Packing of the background into three 4-value records per cell, cell
// (column c, level k) at index c*nz + k: A = (U, V, N2, Ux), then
// (Uy, Uz, Vx, Vy) and (Vz, N2x, N2y, N2z).  The fields arrive level-major
// ([nz][ny][nx]) and the records are column-major, so this is a transpose: a
// workgroup reads a tile of PACK_TC columns x PACK_TK levels of each field in
// runs of consecutive columns, keeps it in LDS, and writes the tile's
// records in runs of consecutive levels.  T is the record precision (the
// single-precision records round each double once).
#pragma once
#include "rt_internal.h"

#define PACK_TC 32
#define PACK_TK 16

template <class T, class T4>
__global__ __launch_bounds__(256) void k_pack(Grid g, Bg<double> b, T4 *__restrict__ A, T4 *__restrict__ G)
{
    __shared__ T tile[12][PACK_TK][PACK_TC + 1];
    const int c0 = blockIdx.x * PACK_TC, k0 = blockIdx.y * PACK_TK;
    const double *src[12] = {b.U, b.V, b.N2, b.Ux, b.Uy, b.Uz, b.Vx, b.Vy, b.Vz, b.N2x, b.N2y, b.N2z};
#pragma unroll
    for (int f = 0; f < 12; f++) {
        for (int e = threadIdx.x; e < PACK_TK * PACK_TC; e += 256) {
            const int c = e % PACK_TC, kk = e / PACK_TC;
            const int col = c0 + c, k = k0 + kk;
            tile[f][kk][c] = (col < g.ncol && k < g.nz) ? (T)src[f][(int64_t)k * g.ncol + col] : (T)0;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < PACK_TK * PACK_TC; e += 256) {
        const int kk = e % PACK_TK, c = e / PACK_TK;
        const int col = c0 + c, k = k0 + kk;
        if (col >= g.ncol || k >= g.nz) continue;
        const int64_t o = (int64_t)col * g.nz + k;
        T4 r;
        r.x = tile[0][kk][c], r.y = tile[1][kk][c], r.z = tile[2][kk][c], r.w = tile[3][kk][c];
        A[o] = r;
        r.x = tile[4][kk][c], r.y = tile[5][kk][c], r.z = tile[6][kk][c], r.w = tile[7][kk][c];
        G[2 * o] = r;
        r.x = tile[8][kk][c], r.y = tile[9][kk][c], r.z = tile[10][kk][c], r.w = tile[11][kk][c];
        G[2 * o + 1] = r;
    }
}

template <class T, class T4>
inline void launch_pack_k(const Grid &g, const Bg<double> &b, T4 *A, T4 *G, hipStream_t s)
{
    const dim3 grid((unsigned)((g.ncol + PACK_TC - 1) / PACK_TC), (unsigned)((g.nz + PACK_TK - 1) / PACK_TK));
    k_pack<T, T4><<<grid, 256, 0, s>>>(g, b, A, G);
}
