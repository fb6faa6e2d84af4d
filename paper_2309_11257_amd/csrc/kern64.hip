// Double-precision kernels: background gradients, load/store, the RK3 step,
// removal tallies, diagnostics and the per-ray deposition payload.
// Built with -ffp-contract=off (see dev64.h).
#include "deposit_common.h"
#include "features_common.h"
#include "dev64.h"
#include "tally_common.h"
#include "pack_common.h"

// ---------------------------------------------------------------------------
// background: centred-difference gradients (periodic in x, and in y on the
// box; one-sided at the vertical ends and the first/last latitude rows)
// ---------------------------------------------------------------------------
// the three gradients of field A at cell c = (i, j, k) of the [nz][ny][nx] layout
__device__ inline void grad3(const Grid &g, const double *A, int64_t c, int i, int j, int k, double &gx, double &gy,
                             double &gz)
{
    const int ip = (i + 1) % g.nx, im = (i + g.nx - 1) % g.nx;
    const int64_t row = (int64_t)g.nx;
    const int64_t plane = (int64_t)g.nx * g.ny;
    gx = (A[c - i + ip] - A[c - i + im]) / (2.0 * g.dx);
    if (g.geometry == RT_CARTESIAN) {
        const int jp = (j + 1) % g.ny, jm = (j + g.ny - 1) % g.ny;
        gy = (A[c + (jp - j) * row] - A[c + (jm - j) * row]) / (2.0 * g.dy);
    } else if (g.ny == 1) {
        gy = 0.0;
    } else if (j == 0) {
        gy = (A[c + row] - A[c]) / g.dy;
    } else if (j == g.ny - 1) {
        gy = (A[c] - A[c - row]) / g.dy;
    } else {
        gy = (A[c + row] - A[c - row]) / (2.0 * g.dy);
    }
    if (g.nz == 1) {
        gz = 0.0;
    } else if (k == 0) {
        gz = (A[c + plane] - A[c]) / g.dz;
    } else if (k == g.nz - 1) {
        gz = (A[c] - A[c - plane]) / g.dz;
    } else {
        gz = (A[c + plane] - A[c - plane]) / (2.0 * g.dz);
    }
}

__global__ void k_gradients(Grid g, const double *U, const double *V, const double *N2, double *out)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int i = (int)(c % g.nx);
    const int j = (int)((c / g.nx) % g.ny);
    const int k = (int)(c / ((int64_t)g.nx * g.ny));
    const double *F[3] = {U, V, N2};
    for (int f = 0; f < 3; f++) {
        double gx, gy, gz;
        grad3(g, F[f], c, i, j, k, gx, gy, gz);
        out[(3 * f + 0) * cells + c] = gx;
        out[(3 * f + 1) * cells + c] = gy;
        out[(3 * f + 2) * cells + c] = gz;
    }
}

// scale-height correction: records (Gamma^2, its x, y, z gradients) by cell,
// column-major like the packed background (cell (column, level) at
// column * nz + level), from the [nz][ny][nx] field; a single-precision
// record rounds each double once
template <class T4>
__global__ void k_gamma_pack(Grid g, const double *G2, T4 *out)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int i = (int)(c % g.nx);
    const int j = (int)((c / g.nx) % g.ny);
    const int k = (int)(c / ((int64_t)g.nx * g.ny));
    double gx, gy, gz;
    grad3(g, G2, c, i, j, k, gx, gy, gz);
    T4 r;
    r.x = G2[c];
    r.y = gx;
    r.z = gy;
    r.w = gz;
    out[((int64_t)j * g.nx + i) * g.nz + k] = r;
}

void launch_gamma_pack(const Grid &g, const double *G2, double4 *out64, float4 *out32, hipStream_t s)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    const unsigned nb = (unsigned)((cells + 255) / 256);
    k_gamma_pack<double4><<<nb, 256, 0, s>>>(g, G2, out64);
    if (out32) k_gamma_pack<float4><<<nb, 256, 0, s>>>(g, G2, out32);
}

__global__ void k_f2(Grid g, const double *f, double *f2, double *f2y)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.ny) return;
    // f^2 per row, then its meridional centred difference
    auto sq = [&](int jj) { const double v = f ? f[jj] : 0.0; return v * v; };
    f2[j] = sq(j);
    double d;
    if (g.geometry == RT_CARTESIAN) {
        const int jp = (j + 1) % g.ny, jm = (j + g.ny - 1) % g.ny;
        d = (sq(jp) - sq(jm)) / (2.0 * g.dy);
    } else if (g.ny == 1) {
        d = 0.0;
    } else if (j == 0) {
        d = (sq(1) - sq(0)) / g.dy;
    } else if (j == g.ny - 1) {
        d = (sq(j) - sq(j - 1)) / g.dy;
    } else {
        d = (sq(j + 1) - sq(j - 1)) / (2.0 * g.dy);
    }
    f2y[j] = d;
}

void launch_gradients64(const Grid &g, const double *U, const double *V, const double *N2, const double *f,
                        double *out12, double *f2, double *f2y, hipStream_t s)
{
    const int64_t cells = (int64_t)g.nx * g.ny * g.nz;
    k_gradients<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(g, U, V, N2, out12);
    k_f2<<<(unsigned)((g.ny + 255) / 256), 256, 0, s>>>(g, f, f2, f2y);
}

// packed column-major records (see rt_internal.h) from the [nz][ny][nx] fields
void launch_pack64(const Grid &g, const Bg<double> &b, double4 *A, double4 *G, hipStream_t s)
{
    launch_pack_k<double, double4>(g, b, A, G, s);
}


// ---------------------------------------------------------------------------
// load / store
// ---------------------------------------------------------------------------
__global__ void k_load64(Grid g, rt_rays in, int64_t n, S64 d, uint32_t *key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y[9] = {in.x[i], in.y[i], in.z[i], in.k[i], in.l[i], in.m[i], in.dx[i], in.dy[i], in.dz[i]};
    const uint32_t kk = d64::post_step(g, Y);
    d.x[i] = Y[0];
    d.y[i] = Y[1];
    d.z[i] = Y[2];
    d.k[i] = Y[3];
    d.l[i] = Y[4];
    d.m[i] = Y[5];
    d.dx[i] = Y[6];
    d.dy[i] = Y[7];
    d.dz[i] = Y[8];
    d.px[i] = in.px[i];
    d.py[i] = in.py[i];
    d.pz[i] = in.pz[i];
    d.n[i] = in.n[i];
    d.id[i] = in.id[i];
    d.W[i] = ((in.n[i] * in.px[i]) * in.py[i]) * in.pz[i];
    key[i] = kk;
}

// next free id = 1 + largest id loaded (ids are non-negative): grid-stride
// maxima, one atomic per wave
__global__ void k_maxid(const int64_t *id, int64_t n, DevCounters *dc)
{
    unsigned long long v = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = (unsigned long long)(id[i] + 1);
        v = c > v ? c : v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v) atomicMax((unsigned long long *)&dc->next_id, v);
}

void launch_maxid(const int64_t *id, int64_t n, DevCounters *dc, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t nb = (n + 255) / 256;
    k_maxid<<<(unsigned)(nb < 2048 ? nb : 2048), 256, 0, s>>>(id, n, dc);
}

void launch_load64(const Grid &g, const rt_rays &in, int64_t n, S64 dst, uint32_t *key, hipStream_t s)
{
    if (n > 0) k_load64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, in, n, dst, key);
}

__global__ void k_store64(S64 st, const uint32_t *perm, const DevCounters *dc, rt_rays o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    o.x[i] = st.x[s];
    o.y[i] = st.y[s];
    o.z[i] = st.z[s];
    o.k[i] = st.k[s];
    o.l[i] = st.l[s];
    o.m[i] = st.m[s];
    o.dx[i] = st.dx[s];
    o.dy[i] = st.dy[s];
    o.dz[i] = st.dz[s];
    const uint32_t h = st.home(s);  // the slot that holds px, py, pz, n and id
    o.px[i] = st.px[h];
    o.py[i] = st.py[h];
    o.pz[i] = st.pz[h];
    o.n[i] = st.n[h];
    o.id[i] = st.id[h];
}

void launch_store64(const Grid &g, S64 src, const uint32_t *perm, const DevCounters *dc, rt_rays out, int64_t bound,
                    hipStream_t s)
{
    (void)g;
    if (bound > 0) k_store64<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(src, perm, dc, out);
}

// ---------------------------------------------------------------------------
// RK3 step (Appendix B: Williamson's low-storage three-stage scheme)
// Reads the current set in sorted order through perm, writes the next
// buffer contiguously, so the state stays grouped by column.
// ---------------------------------------------------------------------------
// One wave per workgroup (a workgroup's slot and stencil box are released as
// soon as its wave ends).  A wave whose volumes share one column first stages
// the background stencil they use into LDS (dev64.h).
#define STEP64_BLOCK 64

template <bool SPH, bool GAM>
__global__ __launch_bounds__(STEP64_BLOCK, 2) void k_step64(Grid g, Bg64P b, S64 src, S64 dst,
                                                            const uint32_t *__restrict__ perm,
                                                            uint32_t *__restrict__ key_out,
                                                            const DevCounters *__restrict__ dc, double dt,
                                                            const uint8_t *__restrict__ frozen,
                                                            const uint32_t *__restrict__ skeys)
{
    const int64_t i = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
    // all lanes take part in the staging (the wave-wide reductions need them)
    const bool valid = i < dc->n_active;
    const uint32_t s = valid ? perm[i] : 0u;
    double Y[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        Y[0] = src.x[s];
        Y[1] = src.y[s];
        Y[2] = src.z[s];
        Y[3] = src.k[s];
        Y[4] = src.l[s];
        Y[5] = src.m[s];
        Y[6] = src.dx[s];
        Y[7] = src.dy[s];
        Y[8] = src.dz[s];
    }
    d64::WBox w;
    {
        // the sorted key of an active slot is its volume's column
        const uint32_t col = valid ? skeys[i] : 0xffffffffu;
        const double q = floor(Y[2] / g.dz);
        const int kc = q >= 0.0 ? (q < (double)(g.nz - 1) ? (int)q : g.nz - 1) : 0;  // NaN gives 0
        const int lane = threadIdx.x & 63;
        const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)col);
        const bool uni = __ballot(valid && col != c0) == 0ull && c0 < (uint32_t)g.ncol;
        const int kmn = wave_min_i(valid ? kc : 0x7fffffff), kmx = wave_max_i(valid ? kc : -1);
        w.ic = (int)(c0 % (uint32_t)g.nx);
        w.jc = (int)(c0 / (uint32_t)g.nx);
        // two levels below and three above the wave's levels hold the faces
        // of most volumes
        w.kbase = max(0, kmn - 2);
        w.L = min(g.nz - 1, kmx + 3) - w.kbase + 1;
        // one wrap corrects a column or row index when the grid has at least two
        w.on = uni && w.L <= WB64_LMAX && g.nx >= 2 && (g.geometry != RT_CARTESIAN || g.ny >= 2);
        if (w.on) {
            // t / L as (t * ceil(2^16 / L)) >> 16, exact for t < 512 and L <= 26
            const int nA = 25 * w.L, nG = 18 * w.L, L9 = 9 * w.L;
            const uint32_t mL = (65536u + (uint32_t)w.L - 1u) / (uint32_t)w.L;
            for (int e = lane; e < nA; e += 64) {
                const int bxy = (int)(((uint32_t)e * mL) >> 16), kk = e - bxy * w.L;
                int ii = w.ic + bxy % 5 - 2, jj = w.jc + bxy / 5 - 2;
                ii += ii < 0 ? g.nx : 0;
                ii -= ii >= g.nx ? g.nx : 0;
                if (g.geometry == RT_CARTESIAN) {
                    jj += jj < 0 ? g.ny : 0;
                    jj -= jj >= g.ny ? g.ny : 0;
                } else {
                    jj = min(max(jj, 0), g.ny - 1);
                }
                d64::wb64_lds[e] = b.A[(jj * g.nx + ii) * g.nz + w.kbase + kk];
            }
            for (int e = lane; e < nG; e += 64) {
                const int r = e >= L9 ? 1 : 0, t = e - r * L9;
                const int bxy = (int)(((uint32_t)t * mL) >> 16), kk = t - bxy * w.L;
                int ii = w.ic + bxy % 3 - 1, jj = w.jc + bxy / 3 - 1;
                ii += ii < 0 ? g.nx : 0;
                ii -= ii >= g.nx ? g.nx : 0;
                if (g.geometry == RT_CARTESIAN) {
                    jj += jj < 0 ? g.ny : 0;
                    jj -= jj >= g.ny ? g.ny : 0;
                } else {
                    jj = min(max(jj, 0), g.ny - 1);
                }
                d64::wb64_lds[WB64_A + r * 9 * WB64_LMAX + t] = b.G[((jj * g.nx + ii) * g.nz + w.kbase + kk) * 2 + r];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (!valid) return;
    double Q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double F[9];
    const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    // volumes in columns handed to the surrogate keep their state this step
    const int nst = (frozen && frozen[skeys[i]]) ? 0 : 3;
#pragma unroll 1
    for (int st = 0; st < nst; st++) {
        d64::rhs<SPH, GAM>(g, b, Y, F, w);
#pragma unroll
        for (int c = 0; c < 9; c++) {
            Q[c] = A[st] * Q[c] + dt * F[c];
            Y[c] = Y[c] + B[st] * Q[c];
        }
    }
    // px, py, pz, n and id stay at their home slot, which is passed on; the
    // wave action is carried with the state (the deposition streams it)
    const uint32_t chm = src.home(s);
    const double cW = src.W[s];
    const uint32_t key = d64::post_step(g, Y);
    dst.x[i] = Y[0];
    dst.y[i] = Y[1];
    dst.z[i] = Y[2];
    dst.k[i] = Y[3];
    dst.l[i] = Y[4];
    dst.m[i] = Y[5];
    dst.dx[i] = Y[6];
    dst.dy[i] = Y[7];
    dst.dz[i] = Y[8];
    dst.hm[i] = chm;
    dst.W[i] = cW;
    key_out[i] = key;
}

void launch_step64(const Grid &g, const Bg64P &b, S64 src, S64 dst, const uint32_t *perm, uint32_t *key_out,
                   const DevCounters *dc, int64_t bound, double dt, const uint8_t *frozen, const uint32_t *skeys,
                   hipStream_t s)
{
    if (bound <= 0) return;
    const unsigned nb = (unsigned)((bound + STEP64_BLOCK - 1) / STEP64_BLOCK);
    const size_t lds = (size_t)WB64_RECS * sizeof(double4);  // the wave's stencil box
    const bool sph = g.geometry == RT_SPHERICAL, gam = b.Gm != nullptr;
    if (sph && gam)
        k_step64<true, true><<<nb, STEP64_BLOCK, lds, s>>>(g, b, src, dst, perm, key_out, dc, dt, frozen, skeys);
    else if (sph)
        k_step64<true, false><<<nb, STEP64_BLOCK, lds, s>>>(g, b, src, dst, perm, key_out, dc, dt, frozen, skeys);
    else if (gam)
        k_step64<false, true><<<nb, STEP64_BLOCK, lds, s>>>(g, b, src, dst, perm, key_out, dc, dt, frozen, skeys);
    else
        k_step64<false, false><<<nb, STEP64_BLOCK, lds, s>>>(g, b, src, dst, perm, key_out, dc, dt, frozen, skeys);
}

// ---------------------------------------------------------------------------
// tallies of volumes removed by the last step (sorted to the end, key =
// ncol + reason) and diagnostics.  One block, fixed assignment and a fixed
// reduction tree: deterministic.
// ---------------------------------------------------------------------------
__device__ inline double W64(const S64 &st, uint32_t s) { return st.W[s]; }

// the wave action of slots 0 .. n - 1 from their n and extents (after an
// operation that rewrote the set; the carried fields are at their slots then)
__global__ void k_refresh_w64(S64 st, int64_t n)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    st.W[s] = ((st.n[s] * st.px[s]) * st.py[s]) * st.pz[s];
}

void launch_refresh_w64(S64 st, int64_t n, hipStream_t s)
{
    if (n > 0) k_refresh_w64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(st, n);
}

struct W64s {
    S64 st;
    __device__ double W(uint32_t slot) const { return W64(st, slot); }
    __device__ int64_t id(uint32_t slot) const { return st.id[st.home(slot)]; }
};

// the carried fields back at the slots: for every sorted position j,
// to.f[perm[j]] = from.f[hm[perm[j]]] (the slots the positions name are
// distinct, and every one of them was written by the step that wrote hm)
__global__ void k_gather_carried64(S64 from, S64 to, const uint32_t *__restrict__ hm,
                                   const uint32_t *__restrict__ perm, const int64_t *__restrict__ n_dev)
{
    const int64_t n = *n_dev;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = perm[j], h = hm[s];
        to.px[s] = from.px[h];
        to.py[s] = from.py[h];
        to.pz[s] = from.pz[h];
        to.n[s] = from.n[h];
        to.id[s] = from.id[h];
    }
}

void launch_gather_carried64(S64 from, S64 to, const uint32_t *hm, const uint32_t *perm, const int64_t *n_dev,
                             int64_t bound, hipStream_t s)
{
    if (bound <= 0) return;
    const int64_t nb = std::min<int64_t>((bound + 255) / 256, 4096);
    k_gather_carried64<<<(unsigned)nb, 256, 0, s>>>(from, to, hm, perm, n_dev);
}

// sort key refined by the level (as in single precision): column key *
// (nz + 1) + floor(z / dz), clamped to 0 .. nz
__global__ void k_levkey64(Grid g, const double *__restrict__ z, uint32_t *__restrict__ key,
                           const DevCounters *__restrict__ dc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_sorted) return;
    const uint32_t k = key[i];
    int l = 0;
    if (k < (uint32_t)g.ncol) {
        const double q = floor(z[i] / g.dz);
        l = q > (double)g.nz ? g.nz : (q >= 0.0 ? (int)q : 0);  // NaN gives 0
    }
    key[i] = k * (uint32_t)(g.nz + 1) + (uint32_t)l;
}

void launch_levkey64(const Grid &g, S64 st, uint32_t *key, const DevCounters *dc, int64_t bound, hipStream_t s)
{
    if (bound <= 0) return;
    k_levkey64<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, st.z, key, dc);
}

void launch_tally64(const Grid &g, S64 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc, double *red,
                    hipStream_t s)
{
    launch_tally_k(g, W64s{st}, perm, skeys, dc, red, s);
}

// sums of W, kW, lW, mW over the active set: per-block partials, then one
// block adds them in order
__global__ void k_stats64_part(S64 st, const uint32_t *perm, const DevCounters *dc, double *part)
{
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    const int64_t n = dc->n_active;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    double v[4] = {0, 0, 0, 0};
    if (i < n) {
        const uint32_t s = perm[i];
        const double W = W64(st, s);
        v[0] = W;
        v[1] = st.k[s] * W;
        v[2] = st.l[s] * W;
        v[3] = st.m[s] * W;
    }
    for (int q = 0; q < 4; q++) sh[q][tid] = v[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int q = 0; q < 4; q++) sh[q][tid] += sh[q][tid + off];
        __syncthreads();
    }
    if (tid < 4) part[4 + (int64_t)blockIdx.x * 4 + tid] = sh[tid][0];
}

__global__ void k_stats_final(double *part, int64_t nblocks)
{
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    double v[4] = {0, 0, 0, 0};
    for (int64_t b = tid; b < nblocks; b += 256)
        for (int q = 0; q < 4; q++) v[q] += part[4 + b * 4 + q];
    for (int q = 0; q < 4; q++) sh[q][tid] = v[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int q = 0; q < 4; q++) sh[q][tid] += sh[q][tid + off];
        __syncthreads();
    }
    if (tid < 4) part[tid] = sh[tid][0];
}

void launch_stats64(S64 st, const uint32_t *perm, const DevCounters *dc, double *red, int64_t bound, hipStream_t s)
{
    const int64_t nb = bound > 0 ? (bound + 255) / 256 : 0;
    if (nb > 0) k_stats64_part<<<(unsigned)nb, 256, 0, s>>>(st, perm, dc, red);
    k_stats_final<<<1, 256, 0, s>>>(red, nb);
}

// ---------------------------------------------------------------------------
// deposition payload: wave action W = N Px Py Pz, intrinsic group velocity at
// the carrier from the dispersion relation (N^2 and f^2 interpolated there)
// ---------------------------------------------------------------------------
// GAM: with the scale-height correction (a separate instantiation, so that
// the form without it carries no extra registers)
template <bool GAM>
struct Pay64 {
    Grid g;
    Bg64P b;
    S64 st;
    double inv_dz;  // unused: the double-precision deposition divides
    static constexpr bool EXACT_LEVELS = true;
    static constexpr int NL = 4, NI = 2;  // horizontal fluxes on levels, vertical on interfaces
    static constexpr int WAVES = 3;
    // a volume's fields as loaded (fetch) and its densities from them (cook)
    struct Raw {
        double x, y, z, k, l, m, Dz, W;
    };
    __device__ void fetch(uint32_t s, Raw &r) const
    {
        r.x = st.x[s];
        r.y = st.y[s];
        r.z = st.z[s];
        r.k = st.k[s];
        r.l = st.l[s];
        r.m = st.m[s];
        r.Dz = st.dz[s];
        r.W = st.W[s];
    }
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        Raw r;
        fetch(s, r);
        cook(r, col, zb, zt, bv);
    }
    __device__ void cook(const Raw &r, int col, double &zb, double &zt, double *bv) const
    {
        (void)col;
        const double x = r.x, y = r.y, z = r.z;
        const double k = r.k, l = r.l, m = r.m, Dz = r.Dz;
        const double W = r.W;
        const d64::Axis ay = d64::axis_y(g, y);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, x), ay, d64::axis_z(g, z));
        const d64::Corners<1> K(b.A, c, 0);
        const double N2 = TRI64(K, z, c);
        const double f2 = d64::row_lerp(b.f2, ay);
        const double kh2 = k * k + l * l;
        const double M2 = m * m + (GAM ? d64::gam2(b, c) : 0.0);
        const double K2 = kh2 + M2;
        const double K4 = K2 * K2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        const double d = N2 - f2;
        const double den = om * K4;
        const double cx = ((k * M2) * d) / den;
        const double cy = ((l * M2) * d) / den;
        const double cz = -(((m * kh2) * d) / den);
        const double sW = W / Dz;
        bv[0] = (cx * k) * sW;
        bv[1] = (cx * l) * sW;
        bv[2] = (cy * k) * sW;
        bv[3] = (cy * l) * sW;
        bv[4] = (cz * k) * sW;
        bv[5] = (cz * l) * sW;
        zb = z - 0.5 * Dz;
        zt = z + 0.5 * Dz;
    }
    // spectral state, wave action and intrinsic vertical group velocity at
    // the carrier (surrogate features)
    __device__ void spec(uint32_t s, double &k, double &l, double &m, double &W, double &cgz, double &z) const
    {
        k = st.k[s];
        l = st.l[s];
        m = st.m[s];
        W = W64(st, s);
        const d64::Axis ay = d64::axis_y(g, st.y[s]);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, st.x[s]), ay, d64::axis_z(g, st.z[s]));
        const d64::Corners<1> K(b.A, c, 0);
        const double N2 = TRI64(K, z, c), f2 = d64::row_lerp(b.f2, ay);
        const double kh2 = k * k + l * l;
        const double M2 = m * m + (GAM ? d64::gam2(b, c) : 0.0);
        const double K2 = kh2 + M2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        cgz = -(((m * kh2) * (N2 - f2)) / (om * (K2 * K2)));
        z = st.z[s];
    }
    __device__ void profile(int col, int k, double &u, double &v, double &n2) const
    {
        const double4 a = b.A[(int64_t)col * g.nz + k];
        u = a.x;
        v = a.y;
        n2 = a.z;
    }
};

void launch_deposit64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, hipStream_t s)
{
    if (b.Gm) {
        Pay64<true> p{g, b, st, 0.0};
        launch_deposit_k(g, p, perm, colstart, flux, s);
    } else {
        Pay64<false> p{g, b, st, 0.0};
        launch_deposit_k(g, p, perm, colstart, flux, s);
    }
}

void launch_features64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s)
{
    const unsigned nb = (unsigned)((g.ncol + 3) / 4);
    if (b.Gm)
        k_features<Pay64<true>><<<nb, 256, 0, s>>>(g, Pay64<true>{g, b, st, 0.0}, perm, colstart, X);
    else
        k_features<Pay64<false>><<<nb, 256, 0, s>>>(g, Pay64<false>{g, b, st, 0.0}, perm, colstart, X);
}
