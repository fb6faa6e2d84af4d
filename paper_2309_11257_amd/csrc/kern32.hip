// Single-precision kernels: load/store between the double-precision
// interface and the FP32 layout (see f32.h), removal tallies, diagnostics,
// the background packing, and the deposition and feature payloads.  The
// wave action W = N Px Py Pz is formed once in double at load and kept in
// double, and every flux sum is accumulated in double.
#include "dev64.h"
#include "tally_common.h"
#include "pack_common.h"
#include "f32.h"
#include "deposit_common.h"
#include "features_common.h"

// ---------------------------------------------------------------------------
// packed single-precision background: A = (U, V, N2, Ux),
// G = (Uy, Uz, Vx, Vy), (Vz, N2x, N2y, N2z) at index col*nz + k
// ---------------------------------------------------------------------------
void launch_pack32(const Grid &g, const Bg<double> &b, float4 *A, float4 *G, hipStream_t s)
{
    launch_pack_k<float, float4>(g, b, A, G, s);
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
__global__ void k_round32(const double *in, float *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void launch_round32(const double *in, float *out, int64_t n, hipStream_t s)
{
    if (n > 0) k_round32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
}

__global__ void k_load32(Grid g, rt_rays in, int64_t n, S32 d, uint32_t *key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y[9] = {in.x[i], in.y[i], in.z[i], in.k[i], in.l[i], in.m[i], in.dx[i], in.dy[i], in.dz[i]};
    const uint32_t kk = d64::post_step(g, Y);
    uint32_t col = 0;
    float xi = 0.0f, eta = 0.0f;
    if (kk < (uint32_t)g.ncol) {
        col = kk;
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        xi = (float)((Y[0] - g.x0) / g.dx - (double)ic);
        eta = (float)((Y[1] - g.y0) / g.dy - (double)jc);
        if (xi >= 1.0f) xi = 0.99999994f;
        if (eta >= 1.0f) eta = 0.99999994f;
    }
    // height as level index + offset in level units
    const double gz = Y[2] / g.dz;
    double fk = floor(gz);
    if (!(fk >= 0.0)) fk = 0.0;
    if (fk > (double)g.nz) fk = (double)g.nz;
    float zeta = (float)(gz - fk);
    if (zeta >= 1.0f) zeta = 0.99999994f;
    d.col[i] = col;
    d.lev[i] = (int32_t)fk;
    d.xi[i] = xi;
    d.eta[i] = eta;
    d.zeta[i] = zeta;
    d.k[i] = (float)Y[3];
    d.l[i] = (float)Y[4];
    d.m[i] = Y[5];
    d.dxi[i] = (float)(Y[6] / g.dx);
    d.deta[i] = (float)(Y[7] / g.dy);
    d.dz[i] = (float)Y[8];
    d.px[i] = (float)in.px[i];
    d.py[i] = (float)in.py[i];
    d.pz[i] = (float)in.pz[i];
    d.W[i] = ((in.n[i] * in.px[i]) * in.py[i]) * in.pz[i];
    d.id[i] = in.id[i];
    key[i] = kk;
}

void launch_load32(const Grid &g, const rt_rays &in, int64_t n, S32 dst, uint32_t *key, hipStream_t s)
{
    if (n > 0) k_load32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, in, n, dst, key);
}

__global__ void k_store32(Grid g, S32 st, const uint32_t *perm, const DevCounters *dc, rt_rays o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    const uint32_t s = perm[i];
    const uint32_t col = st.col[s];
    const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
    o.x[i] = g.x0 + ((double)ic + (double)st.xi[s]) * g.dx;
    o.y[i] = g.y0 + ((double)jc + (double)st.eta[s]) * g.dy;
    o.z[i] = ((double)st.lev[s] + (double)st.zeta[s]) * g.dz;
    o.k[i] = st.k[s];
    o.l[i] = st.l[s];
    o.m[i] = st.m[s];
    o.dx[i] = (double)st.dxi[s] * g.dx;
    o.dy[i] = (double)st.deta[s] * g.dy;
    o.dz[i] = st.dz[s];
    const uint32_t h = st.hm ? st.hm[s] : s;  // the slot that holds px, py, pz and id
    const double px = st.px[h], py = st.py[h], pz = st.pz[h];
    o.px[i] = px;
    o.py[i] = py;
    o.pz[i] = pz;
    o.n[i] = st.W[s] / ((px * py) * pz);
    o.id[i] = st.id[h];
}

void launch_store32(const Grid &g, S32 src, const uint32_t *perm, const DevCounters *dc, rt_rays out, int64_t bound,
                    hipStream_t s)
{
    if (bound > 0) k_store32<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, src, perm, dc, out);
}

// ---------------------------------------------------------------------------
// tallies and diagnostics (deterministic, see kern64.hip and tally_common.h)
// ---------------------------------------------------------------------------
// sort key refined by the level: column key * (nz + 1) + level index, so that
// the sort orders each column's volumes by level and a wave of the step
// covers few levels (removed volumes keep their reason, at level 0)
__global__ void k_levkey32(Grid g, const int32_t *__restrict__ lev, uint32_t *__restrict__ key,
                           const DevCounters *__restrict__ dc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_sorted) return;
    const uint32_t k = key[i];
    const int l = k < (uint32_t)g.ncol ? min(max(lev[i], 0), g.nz) : 0;
    key[i] = k * (uint32_t)(g.nz + 1) + (uint32_t)l;
}

void launch_levkey32(const Grid &g, S32 st, uint32_t *key, const DevCounters *dc, int64_t bound, hipStream_t s)
{
    if (bound <= 0) return;
    k_levkey32<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(g, st.lev, key, dc);
}

struct W32 {
    const double *w;
    const int64_t *ids;
    const uint32_t *hm;  // home slots of the ids (null: the slot itself)
    __device__ double W(uint32_t slot) const { return w[slot]; }
    __device__ int64_t id(uint32_t slot) const { return ids[hm ? hm[slot] : slot]; }
};

void launch_tally32(const Grid &g, S32 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc, double *red,
                    hipStream_t s)
{
    launch_tally_k(g, W32{st.W, st.id, st.hm}, perm, skeys, dc, red, s);
}

// the carried fields back at the slots: for every sorted position j,
// to.f[perm[j]] = from.f[hm[perm[j]]] (the slots the positions name are
// distinct, and every one of them was written by the step that wrote hm)
__global__ void k_gather_carried(S32 from, S32 to, const uint32_t *__restrict__ hm, const uint32_t *__restrict__ perm,
                                 const int64_t *__restrict__ n_dev)
{
    const int64_t n = *n_dev;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = perm[j], h = hm[s];
        to.px[s] = from.px[h];
        to.py[s] = from.py[h];
        to.pz[s] = from.pz[h];
        to.id[s] = from.id[h];
    }
}

void launch_gather_carried(S32 from, S32 to, const uint32_t *hm, const uint32_t *perm, const int64_t *n_dev,
                           int64_t bound, hipStream_t s)
{
    if (bound <= 0) return;
    const int64_t nb = std::min<int64_t>((bound + 255) / 256, 4096);
    k_gather_carried<<<(unsigned)nb, 256, 0, s>>>(from, to, hm, perm, n_dev);
}

__global__ void k_stats32_part(S32 st, const uint32_t *perm, const DevCounters *dc, double *part)
{
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    const int64_t n = dc->n_active;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    double v[4] = {0, 0, 0, 0};
    if (i < n) {
        const uint32_t s = perm[i];
        const double W = st.W[s];
        v[0] = W;
        v[1] = (double)st.k[s] * W;
        v[2] = (double)st.l[s] * W;
        v[3] = (double)st.m[s] * W;
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

__global__ void k_stats32_final(double *part, int64_t nblocks)
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

void launch_stats32(S32 st, const uint32_t *perm, const DevCounters *dc, double *red, int64_t bound, hipStream_t s)
{
    const int64_t nb = bound > 0 ? (bound + 255) / 256 : 0;
    if (nb > 0) k_stats32_part<<<(unsigned)nb, 256, 0, s>>>(st, perm, dc, red);
    k_stats32_final<<<1, 256, 0, s>>>(red, nb);
}

// ---------------------------------------------------------------------------
// deposition payload: single-precision dispersion at the carrier, wave action
// and the flux densities in double
// ---------------------------------------------------------------------------
// GAM: with the scale-height correction (a separate instantiation)
// CAR: N^2, f^2 (and Gamma^2) at the carrier from the state's carrier arrays
// (written by the step that produced the state) instead of interpolated here
template <bool GAM, bool CAR = false>
struct Pay32 {
    G32 g;
    Bg32P b;
    S32 st;
    double zdz;     // level spacing in double
    double inv_dz;  // its reciprocal (level spans of the deposition)
    static constexpr bool EXACT_LEVELS = false;
    static constexpr int NL = 4, NI = 2;  // horizontal fluxes on levels, vertical on interfaces
    static constexpr int WAVES = 4;
    // a volume's fields as loaded (fetch) and its densities from them (cook)
    struct Raw {
        int kc;
        float zeta, k, l, Dz, xi, eta, N2, f2, G2;
        double m, W;
    };
    __device__ void fetch(uint32_t s, Raw &r) const
    {
        r.kc = st.lev[s];
        r.zeta = st.zeta[s];
        r.k = st.k[s];
        r.l = st.l[s];
        r.Dz = st.dz[s];
        r.m = st.m[s];
        r.W = st.W[s];
        if (CAR) {
            r.N2 = st.cn2[s];
            r.f2 = st.cf2[s];
            if (GAM) r.G2 = st.cg2[s];
        } else {
            r.xi = st.xi[s];
            r.eta = st.eta[s];
        }
    }
    __device__ void load(uint32_t s, int col, double &zb, double &zt, double *bv) const
    {
        Raw r;
        fetch(s, r);
        cook(r, col, zb, zt, bv);
    }
    __device__ void cook(const Raw &r, int col, double &zb, double &zt, double *bv) const
    {
        // the wave's column (the slot's own column, by the grouping)
        const int jc = (int)((uint32_t)col / (uint32_t)g.nx), ic = col - jc * g.nx;
        const int kc = r.kc;
        const float zeta = r.zeta;
        const float k = r.k, l = r.l, m = (float)r.m;
        const float Dz = r.Dz;
        float N2, f2, G2 = 0.0f;
        if (CAR) {
            N2 = r.N2;
            f2 = r.f2;
            if (GAM) G2 = r.G2;
        } else {
            f32::n2_f2(g, b, ic, jc, kc, r.xi, r.eta, zeta, N2, f2);
            if (GAM) G2 = f32::gam2_at(g, b, ic, jc, kc, r.xi, r.eta, zeta);
        }
        // group velocity as in the step: one-rounding reciprocal and
        // reciprocal square root
        const float kh2 = k * k + l * l;
        const float M2 = m * m + G2;
        const float invK2 = f32::rcp(kh2 + M2);
        const float rom = f32::rsq((N2 * kh2 + f2 * M2) * invK2);  // 1 / omega_hat
        const float sc = (N2 - f2) * (invK2 * invK2) * rom;
        const double cx = (double)(k * M2 * sc);
        const double cy = (double)(l * M2 * sc);
        const double cz = (double)(-m * kh2 * sc);
        const double sW = r.W * (double)f32::rcp(Dz);
        const double kd = k, ld = l;
        bv[0] = (cx * kd) * sW;
        bv[1] = (cx * ld) * sW;
        bv[2] = (cy * kd) * sW;
        bv[3] = (cy * ld) * sW;
        bv[4] = (cz * kd) * sW;
        bv[5] = (cz * ld) * sW;
        const double zc = ((double)kc + (double)zeta) * zdz;
        zb = zc - 0.5 * (double)Dz;
        zt = zc + 0.5 * (double)Dz;
    }
    // spectral state, wave action and intrinsic vertical group velocity at
    // the carrier (surrogate features)
    __device__ void spec(uint32_t s, double &kd, double &ld, double &md, double &W, double &cgz, double &z) const
    {
        const uint32_t col = st.col[s];
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        float N2, f2;
        f32::n2_f2(g, b, ic, jc, st.lev[s], st.xi[s], st.eta[s], st.zeta[s], N2, f2);
        const float k = st.k[s], l = st.l[s], m = (float)st.m[s];
        const float kh2 = k * k + l * l;
        const float M2 =
            m * m + (GAM ? f32::gam2_at(g, b, ic, jc, st.lev[s], st.xi[s], st.eta[s], st.zeta[s]) : 0.0f);
        const float K2 = kh2 + M2;
        const float om = sqrtf((N2 * kh2 + f2 * M2) / K2);
        const float sc = (N2 - f2) / (K2 * K2) / om;
        kd = k;
        ld = l;
        md = st.m[s];
        W = st.W[s];
        cgz = (double)(-m * kh2 * sc);
        z = ((double)st.lev[s] + (double)st.zeta[s]) * zdz;
    }
    __device__ void profile(int col, int k, double &u, double &v, double &n2) const
    {
        const float4 a = b.A[(int64_t)col * g.nz + k];
        u = a.x;
        v = a.y;
        n2 = a.z;
    }
};

template <bool GAM, bool CAR>
static void deposit32_with(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                           double *flux, hipStream_t s)
{
    Pay32<GAM, CAR> p{f32::make_g32(g), b, st, g.dz, 1.0 / g.dz};
    launch_deposit_k(g, p, perm, colstart, flux, s);
}

void launch_deposit32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, bool car, hipStream_t s)
{
    if (b.Gm)
        car ? deposit32_with<true, true>(g, b, st, perm, colstart, flux, s)
            : deposit32_with<true, false>(g, b, st, perm, colstart, flux, s);
    else
        car ? deposit32_with<false, true>(g, b, st, perm, colstart, flux, s)
            : deposit32_with<false, false>(g, b, st, perm, colstart, flux, s);
}

void launch_features32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s)
{
    const unsigned nb = (unsigned)((g.ncol + 3) / 4);
    const G32 h = f32::make_g32(g);
    if (b.Gm)
        k_features<Pay32<true>><<<nb, 256, 0, s>>>(g, Pay32<true>{h, b, st, g.dz, 1.0 / g.dz}, perm, colstart, X);
    else
        k_features<Pay32<false>><<<nb, 256, 0, s>>>(g, Pay32<false>{h, b, st, g.dz, 1.0 / g.dz}, perm, colstart, X);
}
