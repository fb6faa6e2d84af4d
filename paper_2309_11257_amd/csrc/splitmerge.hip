// Vertical splitting, per-cell merge and per-column cap (rt_split_merge).
//
// Sequence: (1) compact the active set into the spare buffer in column order;
// (2) split: count the pieces of every volume taller than alpha dz, order the
// splitting volumes by id (two stable 32-bit radix sorts), give the new
// pieces consecutive ids in that order (exclusive scan), write the pieces;
// (3) regroup by column; (4) merge per 3-D cell or cap per column, one
// workgroup per over-full cell/column: its volumes are ordered in LDS
// (bitonic sort), and one lane walks the order exactly as the reference
// rule does, so the result does not depend on scheduling; (5) rekey and
// regroup.  Double-precision arithmetic here is built with
// -ffp-contract=off and follows the same operation order as the split and
// merge rules are written (halving by 0.5, W-weighted means, bounding hulls).
#include "dev64.h"

#define SM_MAX_CELL 2048  // records of one cell/column sorted in LDS (24 B each)

// ---------------------------------------------------------------------------
// common helpers
// ---------------------------------------------------------------------------
__device__ inline int octant_of(double k, double l)
{
    const int q = (k >= 0.0) ? (l >= 0.0 ? 0 : 3) : (l >= 0.0 ? 1 : 2);
    const int big_l = fabs(l) > fabs(k);
    const int off = (q == 0 || q == 2) ? big_l : !big_l;
    return 2 * q + off;
}

// spectral group: azimuth octant of (k, l), sign of m, binary exponent of |m|
__device__ inline uint64_t group_of(double k, double l, double m)
{
    int e;
    frexp(fabs(m), &e);
    const int64_t gk = ((int64_t)(octant_of(k, l) * 2 + (m < 0.0 ? 0 : 1)) << 16) + (int64_t)(e + 4096);
    return (uint64_t)gk;
}

// uniform view of one ray volume in double precision, whatever the storage
struct RayD {
    double x, y, z, k, l, m, dx, dy, dz, px, py, pz, W, n;
    int64_t id;
};

__device__ inline double metric_x(const Grid &g, double y, double z, double D)
{
    return g.geometry == RT_CARTESIAN ? D : ((g.a + z) * cos(y)) * D;
}
__device__ inline double metric_y(const Grid &g, double z, double D)
{
    return g.geometry == RT_CARTESIAN ? D : (g.a + z) * D;
}

// --- double-precision storage ----------------------------------------------
struct IO64 {
    S64 s;
    const double *f2r;            // f^2 by latitude row
    const double4 *Gm = nullptr;  // Gamma^2 records (wave energy), null when Gamma = 0
    __device__ RayD get(const Grid &g, uint32_t i) const
    {
        RayD r;
        r.x = s.x[i];
        r.y = s.y[i];
        r.z = s.z[i];
        r.k = s.k[i];
        r.l = s.l[i];
        r.m = s.m[i];
        r.dx = s.dx[i];
        r.dy = s.dy[i];
        r.dz = s.dz[i];
        r.px = s.px[i];
        r.py = s.py[i];
        r.pz = s.pz[i];
        r.W = ((s.n[i] * s.px[i]) * s.py[i]) * s.pz[i];
        r.n = s.n[i];
        r.id = s.id[i];
        (void)g;
        return r;
    }
    // set_n: N = W / (Px Py Pz) (merge); otherwise N is carried unchanged
    __device__ void put(const Grid &g, uint32_t i, const RayD &r, bool set_n) const
    {
        (void)g;
        s.x[i] = r.x;
        s.y[i] = r.y;
        s.z[i] = r.z;
        s.k[i] = r.k;
        s.l[i] = r.l;
        s.m[i] = r.m;
        s.dx[i] = r.dx;
        s.dy[i] = r.dy;
        s.dz[i] = r.dz;
        s.px[i] = r.px;
        s.py[i] = r.py;
        s.pz[i] = r.pz;
        s.n[i] = set_n ? r.W / ((r.px * r.py) * r.pz) : r.n;
        s.id[i] = r.id;
    }
    __device__ int64_t get_id(uint32_t i) const { return s.id[i]; }
    __device__ void copy2(const IO64 &d, uint32_t from, uint32_t to) const
    {
        d.s.x[to] = s.x[from];
        d.s.y[to] = s.y[from];
        d.s.z[to] = s.z[from];
        d.s.k[to] = s.k[from];
        d.s.l[to] = s.l[from];
        d.s.m[to] = s.m[from];
        d.s.dx[to] = s.dx[from];
        d.s.dy[to] = s.dy[from];
        d.s.dz[to] = s.dz[from];
        d.s.px[to] = s.px[from];
        d.s.py[to] = s.py[from];
        d.s.pz[to] = s.pz[from];
        d.s.n[to] = s.n[from];
        d.s.id[to] = s.id[from];
    }
    __device__ double height(const Grid &g, uint32_t i) const
    {
        (void)g;
        return s.z[i];
    }
    __device__ double dzv(uint32_t i) const { return s.dz[i]; }
    __device__ double pzv(uint32_t i) const { return s.pz[i]; }
    __device__ double wv(uint32_t i) const { return ((s.n[i] * s.px[i]) * s.py[i]) * s.pz[i]; }
    // a split piece: N is unchanged, so W follows from Pz
    __device__ void set_piece(const Grid &g, uint32_t i, double z, double D, double P, double W, int64_t id) const
    {
        (void)g;
        (void)W;
        s.z[i] = z;
        s.dz[i] = D;
        s.pz[i] = P;
        s.id[i] = id;
    }
    __device__ uint32_t column(const Grid &g, uint32_t i) const { return (uint32_t)d64::column_of(g, s.x[i], s.y[i]); }
    __device__ void rewrap(const Grid &g, uint32_t i) const
    {
        double x = s.x[i], y = s.y[i];
        d64::wrap(x, g.x0, g.Lx);
        if (g.geometry == RT_CARTESIAN) d64::wrap(y, g.y0, g.Ly);
        s.x[i] = x;
        s.y[i] = y;
    }
    __device__ double energy(const Grid &g, const double4 *bA, uint32_t i) const
    {
        const d64::Axis ay = d64::axis_y(g, s.y[i]);
        const d64::Cell c = d64::cell_of(g, d64::axis_x(g, s.x[i]), ay, d64::axis_z(g, s.z[i]));
        const d64::Corners<1> K(bA, c, 0);
        const double N2 = TRI64(K, z, c), f2 = d64::row_lerp(f2r, ay);
        const double k = s.k[i], l = s.l[i], m = s.m[i];
        const double kh2 = k * k + l * l;
        const double M2 = m * m + d64::gam2(Gm, c);
        const double K2 = kh2 + M2;
        const double om = d64::omega_hat(N2, f2, kh2, M2, K2);
        return om * (((s.n[i] * s.px[i]) * s.py[i]) * s.pz[i]);
    }
};

// --- single-precision storage (positions as cell + offset) -----------------
struct IO32 {
    S32 s;
    const float *f2r;            // f^2 by latitude row
    const float4 *Gm = nullptr;  // Gamma^2 records (wave energy), null when Gamma = 0
    __device__ RayD get(const Grid &g, uint32_t i) const
    {
        RayD r;
        const uint32_t col = s.col[i];
        const int ic = (int)(col % (uint32_t)g.nx), jc = (int)(col / (uint32_t)g.nx);
        r.x = g.x0 + ((double)ic + (double)s.xi[i]) * g.dx;
        r.y = g.y0 + ((double)jc + (double)s.eta[i]) * g.dy;
        r.z = ((double)s.lev[i] + (double)s.zeta[i]) * g.dz;
        r.k = s.k[i];
        r.l = s.l[i];
        r.m = s.m[i];
        r.dx = (double)s.dxi[i] * g.dx;
        r.dy = (double)s.deta[i] * g.dy;
        r.dz = s.dz[i];
        r.px = s.px[i];
        r.py = s.py[i];
        r.pz = s.pz[i];
        r.W = s.W[i];
        r.n = 0.0;
        r.id = s.id[i];
        return r;
    }
    __device__ void put(const Grid &g, uint32_t i, const RayD &r, bool set_n) const
    {
        (void)set_n;
        double fi = floor((r.x - g.x0) / g.dx), fj = floor((r.y - g.y0) / g.dy);
        fi = fmin(fmax(fi, 0.0), (double)(g.nx - 1));
        fj = fmin(fmax(fj, 0.0), (double)(g.ny - 1));
        double fk = floor(r.z / g.dz);
        fk = fmin(fmax(fk, 0.0), (double)g.nz);
        s.col[i] = (uint32_t)((int)fj * g.nx + (int)fi);
        s.xi[i] = (float)((r.x - g.x0) / g.dx - fi);
        s.eta[i] = (float)((r.y - g.y0) / g.dy - fj);
        s.lev[i] = (int32_t)fk;
        s.zeta[i] = (float)(r.z / g.dz - fk);
        s.k[i] = (float)r.k;
        s.l[i] = (float)r.l;
        s.m[i] = r.m;
        s.dxi[i] = (float)(r.dx / g.dx);
        s.deta[i] = (float)(r.dy / g.dy);
        s.dz[i] = (float)r.dz;
        s.px[i] = (float)r.px;
        s.py[i] = (float)r.py;
        s.pz[i] = (float)r.pz;
        s.W[i] = r.W;
        s.id[i] = r.id;
    }
    __device__ int64_t get_id(uint32_t i) const { return s.id[i]; }
    __device__ void copy2(const IO32 &d, uint32_t from, uint32_t to) const
    {
        d.s.col[to] = s.col[from];
        d.s.lev[to] = s.lev[from];
        d.s.xi[to] = s.xi[from];
        d.s.eta[to] = s.eta[from];
        d.s.zeta[to] = s.zeta[from];
        d.s.k[to] = s.k[from];
        d.s.l[to] = s.l[from];
        d.s.m[to] = s.m[from];
        d.s.dxi[to] = s.dxi[from];
        d.s.deta[to] = s.deta[from];
        d.s.dz[to] = s.dz[from];
        d.s.px[to] = s.px[from];
        d.s.py[to] = s.py[from];
        d.s.pz[to] = s.pz[from];
        d.s.W[to] = s.W[from];
        d.s.id[to] = s.id[from];
    }
    __device__ double height(const Grid &g, uint32_t i) const { return ((double)s.lev[i] + (double)s.zeta[i]) * g.dz; }
    __device__ double dzv(uint32_t i) const { return s.dz[i]; }
    __device__ double pzv(uint32_t i) const { return s.pz[i]; }
    __device__ double wv(uint32_t i) const { return s.W[i]; }
    __device__ void set_piece(const Grid &g, uint32_t i, double z, double D, double P, double W, int64_t id) const
    {
        double fk = floor(z / g.dz);
        fk = fmin(fmax(fk, 0.0), (double)g.nz);
        s.lev[i] = (int32_t)fk;
        s.zeta[i] = (float)(z / g.dz - fk);
        s.dz[i] = (float)D;
        s.pz[i] = (float)P;
        s.W[i] = W;
        s.id[i] = id;
    }
    __device__ uint32_t column(const Grid &g, uint32_t i) const { (void)g; return s.col[i]; }
    __device__ void rewrap(const Grid &g, uint32_t i) const { (void)g; (void)i; }
    // wave energy from the single-precision background (N2 from the packed A
    // record, f2 by row), in double
    __device__ double energy(const Grid &g, const float4 *bA, uint32_t i) const
    {
        const RayD r = get(g, i);
        d64::Cell c;
        d64::locate(g, r.x, r.y, r.z, c);
        const int o[8] = {c.c00 + c.k0, c.c01 + c.k0, c.c10 + c.k0, c.c11 + c.k0,
                          c.c00 + c.k1, c.c01 + c.k1, c.c10 + c.k1, c.c11 + c.k1};
        double vz[8];
        for (int q = 0; q < 8; q++) vz[q] = bA[o[q]].z;
        auto tri = [&](const double *v) {
            const double c00 = v[0] + c.wx * (v[1] - v[0]), c10 = v[2] + c.wx * (v[3] - v[2]);
            const double c01 = v[4] + c.wx * (v[5] - v[4]), c11 = v[6] + c.wx * (v[7] - v[6]);
            const double c0 = c00 + c.wy * (c10 - c00), c1 = c01 + c.wy * (c11 - c01);
            return c0 + c.wz * (c1 - c0);
        };
        double4 A;
        A.z = tri(vz);
        const int j0 = (c.c00 / g.nz) / g.nx, j1 = (c.c10 / g.nz) / g.nx;
        A.w = (double)f2r[j0] + c.wy * ((double)f2r[j1] - (double)f2r[j0]);
        double G2 = 0.0;
        if (Gm) {
            double vg[8];
            for (int q = 0; q < 8; q++) vg[q] = Gm[o[q]].x;
            G2 = tri(vg);
        }
        const double kh2 = r.k * r.k + r.l * r.l;
        const double M2 = r.m * r.m + G2;
        const double K2 = kh2 + M2;
        return d64::omega_hat(A.z, A.w, kh2, M2, K2) * r.W;
    }
};

// ---------------------------------------------------------------------------
// compaction of the active set into the spare buffer, in column order
// ---------------------------------------------------------------------------
template <class IO>
__global__ void k_compact(IO src, IO dst, const uint32_t *perm, const uint32_t *skeys, uint32_t *key_dst,
                          const DevCounters *dc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dc->n_active) return;
    src.copy2(dst, perm[i], (uint32_t)i);
    key_dst[i] = skeys[i];
}

// ---------------------------------------------------------------------------
// split
// ---------------------------------------------------------------------------
__device__ inline uint32_t pieces_of(double Dz, double thr)
{
    double D = Dz;
    uint32_t p = 1;
    while (D > thr && p < 64) {
        D = 0.5 * D;
        p *= 2;
    }
    return p;
}

template <class IO>
__global__ void k_split_count(IO io, const uint32_t *key, int64_t n, int ncol, double thr, uint32_t *extra,
                              uint32_t *idlo, uint32_t *idhi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool act = key[i] < (uint32_t)ncol;
    extra[i] = (act && thr > 0.0) ? pieces_of(io.dzv((uint32_t)i), thr) - 1u : 0u;
    const int64_t id = io.get_id((uint32_t)i);
    idlo[i] = (uint32_t)((uint64_t)id & 0xffffffffull);
    idhi[i] = (uint32_t)((uint64_t)id >> 32);
}

__global__ void k_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_split_total(const uint32_t *ex_sorted_scan, const uint32_t *ex_sorted, int64_t n, DevCounters *dc)
{
    dc->split_extra = n > 0 ? (int64_t)ex_sorted_scan[n - 1] + (int64_t)ex_sorted[n - 1] : 0;
}

// r-th splitting volume in id order: lowest piece stays in its slot, the
// others go to slots n + off[r] + (q - 1) with ids next_id + off[r] + (q - 1).
// Piece q's height follows the halving tree from the root: at each level the
// lower half is at z - D/4 and the upper at z + D/4, with D and Pz halved.
// Pieces are full copies of the parent except for (z, Dz, Pz, W, id); the
// parent slot is rewritten last.
template <class IO>
__global__ void k_split_write(IO io, const Grid g, uint32_t *key, const uint32_t *pid, const uint32_t *off,
                              const uint32_t *ex, int64_t n, int64_t next_id)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t extra = ex[r];
    if (extra == 0) return;
    const uint32_t s = pid[r];
    const uint32_t p = extra + 1;
    int levels = 0;
    while ((1u << levels) < p) levels++;
    const double z0 = io.height(g, s), D0 = io.dzv(s), P0 = io.pzv(s), W0 = io.wv(s);
    const int64_t id0 = io.get_id(s);
    const uint32_t pkey = key[s];
    for (int qq = (int)p - 1; qq >= 0; qq--) {
        const uint32_t q = (uint32_t)qq;
        double z = z0, D = D0, P = P0, Wc = W0;
        for (int t = 0; t < levels; t++) {
            const uint32_t bit = (q >> (levels - 1 - t)) & 1u;
            z = bit ? z + 0.25 * D : z - 0.25 * D;
            D = 0.5 * D;
            P = 0.5 * P;
            Wc = 0.5 * Wc;
        }
        uint32_t dst = s;
        int64_t id = id0;
        if (q > 0) {
            dst = (uint32_t)(n + (int64_t)off[r] + (int64_t)(q - 1));
            id = next_id + (int64_t)off[r] + (int64_t)(q - 1);
            io.copy2(io, s, dst);
            key[dst] = pkey;
        }
        io.set_piece(g, dst, z, D, P, Wc, id);
    }
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
template <class IO>
__global__ void k_rekey(IO io, const Grid g, uint32_t *key, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (key[i] >= (uint32_t)g.ncol) return;  // removed volumes keep their reason
    io.rewrap(g, (uint32_t)i);
    key[i] = io.column(g, (uint32_t)i);
}

template <class IO>
__global__ void k_key3(IO io, const Grid g, const uint32_t *key, uint32_t *key3, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t ncell = (uint32_t)g.ncol * (uint32_t)g.nz;
    if (key[i] >= (uint32_t)g.ncol) {
        key3[i] = ncell;
        return;
    }
    double fk = floor(io.height(g, (uint32_t)i) / g.dz);
    if (fk < 0.0) fk = 0.0;
    if (fk > (double)(g.nz - 1)) fk = (double)(g.nz - 1);
    key3[i] = key[i] * (uint32_t)g.nz + (uint32_t)fk;
}

// over-full segments of sorted keys: (start, count) appended to a list
__global__ void k_overfull(const uint32_t *skeys, int64_t n, uint32_t limit_key, int32_t nmax, uint32_t *list,
                           uint32_t *nlist, uint32_t *maxcount)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = skeys[p];
    if (k >= limit_key) return;
    if (p > 0 && skeys[p - 1] == k) return;
    int64_t lo = p, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skeys[mid] <= k)
            lo = mid + 1;
        else
            hi = mid;
    }
    const uint32_t cnt = (uint32_t)(lo - p);
    if ((int32_t)cnt <= nmax) return;
    const uint32_t at = atomicAdd(nlist, 1u);
    list[2 * at] = (uint32_t)p;
    list[2 * at + 1] = cnt;
    atomicMax(maxcount, cnt);
}

// ---------------------------------------------------------------------------
// block bitonic sort of (k1, k2, payload) records in LDS, ascending
// ---------------------------------------------------------------------------
__device__ inline bool rec_less(uint64_t a1, uint64_t a2, uint64_t b1, uint64_t b2)
{
    return a1 < b1 || (a1 == b1 && a2 < b2);
}

__device__ void block_bitonic(uint64_t *k1, uint64_t *k2, uint32_t *pl, int N)
{
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < N / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const bool sw = up ? rec_less(k1[hi], k2[hi], k1[lo], k2[lo]) : rec_less(k1[lo], k2[lo], k1[hi], k2[hi]);
                if (sw) {
                    const uint64_t a = k1[lo], b = k2[lo];
                    const uint32_t c = pl[lo];
                    k1[lo] = k1[hi];
                    k2[lo] = k2[hi];
                    pl[lo] = pl[hi];
                    k1[hi] = a;
                    k2[hi] = b;
                    pl[hi] = c;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// merge two volumes (survivor a): summed wave action, W-weighted carrier
// position and wavevector, physical and spectral extents spanning both
// ---------------------------------------------------------------------------
__device__ inline void merge_pair(const Grid &g, RayD &a, const RayD &b)
{
    const double Wa = a.W, Wb = b.W, W = Wa + Wb;
    const double dka = a.px / metric_x(g, a.y, a.z, a.dx);
    const double dkb = b.px / metric_x(g, b.y, b.z, b.dx);
    const double dla = a.py / metric_y(g, a.z, a.dy);
    const double dlb = b.py / metric_y(g, b.z, b.dy);
    const double dma = a.pz / a.dz, dmb = b.pz / b.dz;
    auto hull = [](double ca, double da, double cb, double db) {
        const double la = ca - 0.5 * da, lb = cb - 0.5 * db;
        const double ha = ca + 0.5 * da, hb = cb + 0.5 * db;
        const double lo = la < lb ? la : lb;
        const double hi = ha > hb ? ha : hb;
        return hi - lo;
    };
    const double x = (a.x * Wa + b.x * Wb) / W;
    const double y = (a.y * Wa + b.y * Wb) / W;
    const double z = (a.z * Wa + b.z * Wb) / W;
    const double k = (a.k * Wa + b.k * Wb) / W;
    const double l = (a.l * Wa + b.l * Wb) / W;
    const double m = (a.m * Wa + b.m * Wb) / W;
    const double Dx = hull(a.x, a.dx, b.x, b.dx);
    const double Dy = hull(a.y, a.dy, b.y, b.dy);
    const double Dz = hull(a.z, a.dz, b.z, b.dz);
    const double Dk = hull(a.k, dka, b.k, dkb);
    const double Dl = hull(a.l, dla, b.l, dlb);
    const double Dm = hull(a.m, dma, b.m, dmb);
    a.x = x;
    a.y = y;
    a.z = z;
    a.k = k;
    a.l = l;
    a.m = m;
    a.dx = Dx;
    a.dy = Dy;
    a.dz = Dz;
    a.px = metric_x(g, y, z, Dx) * Dk;
    a.py = metric_y(g, z, Dy) * Dl;
    a.pz = Dz * Dm;
    a.W = W;
}

// one workgroup per over-full cell; records sorted by (group, id)
template <class IO>
__global__ __launch_bounds__(256) void k_merge_cells(IO io, const Grid g, const uint32_t *perm3, const uint32_t *list,
                                                     uint32_t *key, int32_t nmax, DevCounters *dc)
{
    extern __shared__ unsigned char sm_smem[];
    const uint32_t start = list[2 * blockIdx.x], cnt = list[2 * blockIdx.x + 1];
    int N = 1;
    while ((uint32_t)N < cnt) N <<= 1;
    uint64_t *k1 = (uint64_t *)sm_smem;
    uint64_t *k2 = k1 + N;
    uint32_t *pl = (uint32_t *)(k2 + N);
    uint32_t *alive = pl + N;  // by position in the cell's original order
    __shared__ int s_count, s_merged, s_done, s_np;
    for (int q = threadIdx.x; q < (int)cnt; q += blockDim.x) alive[q] = 1u;
    if (threadIdx.x == 0) {
        s_count = (int)cnt;
        s_merged = 0;
        s_done = 0;
    }
    __syncthreads();
    while (true) {
        if (s_done || s_count <= nmax) break;
        // records of the surviving volumes, keyed by (group, id)
        for (int q = threadIdx.x; q < N; q += blockDim.x) {
            if (q < (int)cnt && alive[q]) {
                const uint32_t s = perm3[start + q];
                const RayD r = io.get(g, s);
                k1[q] = group_of(r.k, r.l, r.m);
                k2[q] = (uint64_t)r.id;
                pl[q] = (uint32_t)q;
            } else {
                k1[q] = ~0ull;
                k2[q] = ~0ull;
                pl[q] = 0xffffffffu;
            }
        }
        __syncthreads();
        block_bitonic(k1, k2, pl, N);
        // the pairs, chosen in sorted order as a sequential pass would: a
        // record and the next one of the same group, until the cell holds
        // nmax volumes (if no two records share a group, neighbours in
        // sorted order); the list goes over the sorted ids, no longer needed
        if (threadIdx.x == 0) {
            int m_ = 0;
            while (m_ < N && pl[m_] != 0xffffffffu) m_++;
            const int want = s_count - nmax;
            int np = 0;
            for (int q = 0; q + 1 < m_ && np < want;) {
                if (k1[q] == k1[q + 1]) {
                    k2[np++] = (uint64_t)q;
                    q += 2;
                } else {
                    q += 1;
                }
            }
            if (np == 0)
                for (int q = 0; q + 1 < m_ && np < want; q += 2) k2[np++] = (uint64_t)q;
            s_np = np;
        }
        __syncthreads();
        // the pairs are disjoint: merged in parallel
        const int np = s_np;
        for (int t = threadIdx.x; t < np; t += blockDim.x) {
            const int q = (int)k2[t];
            const uint32_t sa = perm3[start + pl[q]], sb = perm3[start + pl[q + 1]];
            RayD a = io.get(g, sa);
            const RayD b = io.get(g, sb);
            merge_pair(g, a, b);
            io.put(g, sa, a, true);
            key[sb] = (uint32_t)(g.ncol + RK_MERGED);
            alive[pl[q + 1]] = 0u;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (np == 0) s_done = 1;
            s_count -= np;
            s_merged += np;
        }
        __threadfence();
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)&dc->n_merged, (unsigned long long)s_merged);
}

// one workgroup per over-full column; remove the lowest wave energies
template <class IO, class AT>
__global__ __launch_bounds__(256) void k_cap_columns(IO io, const Grid g, const AT *bA, const uint32_t *perm,
                                                     const uint32_t *list, uint32_t *key, int32_t nmax)
{
    extern __shared__ unsigned char sm_smem[];
    const uint32_t start = list[2 * blockIdx.x], cnt = list[2 * blockIdx.x + 1];
    int N = 1;
    while ((uint32_t)N < cnt) N <<= 1;
    uint64_t *k1 = (uint64_t *)sm_smem;
    uint64_t *k2 = k1 + N;
    uint32_t *pl = (uint32_t *)(k2 + N);
    for (int q = threadIdx.x; q < N; q += blockDim.x) {
        if (q < (int)cnt) {
            const uint32_t s = perm[start + q];
            const double E = io.energy(g, bA, s);
            k1[q] = (uint64_t)__double_as_longlong(E);  // E > 0: bit order = numeric order
            k2[q] = ~(uint64_t)io.get_id(s);            // among equal energies the larger id first
            pl[q] = s;
        } else {
            k1[q] = ~0ull;
            k2[q] = ~0ull;
            pl[q] = 0xffffffffu;
        }
    }
    __syncthreads();
    block_bitonic(k1, k2, pl, N);
    for (int q = threadIdx.x; q < (int)cnt - nmax; q += blockDim.x) key[pl[q]] = (uint32_t)(g.ncol + RK_CAPPED);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int bits_for(uint64_t maxkey)
{
    int b = 0;
    while (b < 64 && (1ull << b) <= maxkey) b++;
    return b;
}

template <class IO, class AT>
static rt_status split_merge_impl(rt_ctx ctx, IO cur_io, IO other_io, const AT *bA, double alpha, int32_t nmax,
                                  int32_t mode)
{
    const Grid &g = ctx->g;
    hipStream_t st = ctx->stream;
    DevCounters h;
    HIP_OK(hipMemcpyAsync(&h, ctx->dc, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    int64_t n = h.n_active;
    const int64_t cap = ctx->cap;
    const unsigned T = 256;
    auto nb = [&](int64_t m) { return (unsigned)((m + T - 1) / T > 0 ? (m + T - 1) / T : 1); };
    rt_status result = RT_OK;

    // scratch carved from ctx->sm (uint32): extra | idlo | idhi | exs | offs | key3 | list | small
    uint32_t *extra = ctx->sm, *idlo = extra + cap, *idhi = idlo + cap, *exs = idhi + cap, *offs = exs + cap;
    uint32_t *key3 = offs + cap, *list = key3 + cap, *small = list + 2 * cap;  // small: nlist, maxcount
    uint32_t *parts = small + 8;

    // (1) compaction into the spare buffer, in column order
    const int nxt = 1 - ctx->cur;
    if (n > 0) k_compact<IO><<<nb(n), T, 0, st>>>(cur_io, other_io, ctx->perm, ctx->skeys, ctx->key[nxt], ctx->dc);
    ctx->cur = nxt;
    IO io = other_io;
    uint32_t *key = ctx->key[ctx->cur];

    // (2) split
    if (alpha > 0.0 && n > 0) {
        const double thr = alpha * g.dz;
        k_split_count<IO><<<nb(n), T, 0, st>>>(io, key, n, g.ncol, thr, extra, idlo, idhi);
        launch_set_sorted(ctx->dc, n, st);
        // slots in id order: stable sort on the low word, then on the high word
        radix_sort(idlo, nullptr, ctx->skeys, ctx->perm, ctx->tk, ctx->tv, ctx->hist, &ctx->dc->n_sorted, n, 32, st);
        const uint32_t *pid = ctx->perm;
        if ((uint64_t)h.next_id > 0xffffffffull) {
            k_gather_u32<<<nb(n), T, 0, st>>>(idhi, ctx->perm, idlo, n);
            radix_sort(idlo, ctx->perm, ctx->skeys, exs, ctx->tk, ctx->tv, ctx->hist, &ctx->dc->n_sorted, n,
                       bits_for((uint64_t)h.next_id >> 32), st);
            HIP_OK(hipMemcpyAsync(ctx->perm, exs, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
        }
        k_gather_u32<<<nb(n), T, 0, st>>>(extra, pid, exs, n);
        HIP_OK(hipMemcpyAsync(offs, exs, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
        scan_u32(offs, n, parts, st);
        k_split_total<<<1, 1, 0, st>>>(offs, exs, n, ctx->dc);
        int64_t total = 0;
        HIP_OK(hipMemcpyAsync(&total, &ctx->dc->split_extra, sizeof(total), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (n + total > cap) {
            result = rt_fail(ctx, RT_E_CAPACITY, "split needs %lld ray volumes, capacity %lld", (long long)(n + total),
                             (long long)cap);
        } else if (total > 0) {
            k_split_write<IO><<<nb(n), T, 0, st>>>(io, g, key, pid, offs, exs, n, h.next_id);
            h.next_id += total;
            h.n_split += total;
            HIP_OK(hipMemcpyAsync(&ctx->dc->next_id, &h.next_id, sizeof(int64_t), hipMemcpyHostToDevice, st));
            HIP_OK(hipMemcpyAsync(&ctx->dc->n_split, &h.n_split, sizeof(int64_t), hipMemcpyHostToDevice, st));
            n += total;
        }
    }

    // (3) merge per 3-D cell or cap per column
    if (result == RT_OK && n > 0 && (mode == RT_MERGE || mode == RT_CAP)) {
        HIP_OK(hipMemsetAsync(small, 0, 8 * sizeof(uint32_t), st));
        launch_set_sorted(ctx->dc, n, st);
        const uint32_t *ord;
        if (mode == RT_MERGE) {
            const uint64_t ncell = (uint64_t)g.ncol * (uint64_t)g.nz;
            k_key3<IO><<<nb(n), T, 0, st>>>(io, g, key, key3, n);
            radix_sort(key3, nullptr, ctx->skeys, ctx->perm, ctx->tk, ctx->tv, ctx->hist, &ctx->dc->n_sorted, n,
                       bits_for(ncell), st);
            k_overfull<<<nb(n), T, 0, st>>>(ctx->skeys, n, (uint32_t)ncell, nmax, list, small, small + 1);
        } else {
            k_rekey<IO><<<nb(n), T, 0, st>>>(io, g, key, n);
            radix_sort(key, nullptr, ctx->skeys, ctx->perm, ctx->tk, ctx->tv, ctx->hist, &ctx->dc->n_sorted, n,
                       bits_for((uint64_t)g.ncol + RK_NREASON), st);
            k_overfull<<<nb(n), T, 0, st>>>(ctx->skeys, n, (uint32_t)g.ncol, nmax, list, small, small + 1);
        }
        ord = ctx->perm;
        uint32_t hs[2];
        HIP_OK(hipMemcpyAsync(hs, small, sizeof(hs), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (hs[0] > 0) {
            if (hs[1] > SM_MAX_CELL) {
                result = rt_fail(ctx, RT_E_UNSUPPORTED, "%s holds %u ray volumes; at most %d are handled",
                                 mode == RT_MERGE ? "a cell" : "a column", hs[1], SM_MAX_CELL);
            } else {
                int N = 1;
                while ((uint32_t)N < hs[1]) N <<= 1;
                const size_t smem = (size_t)N * (8 + 8 + 4 + 4);
                if (mode == RT_MERGE)
                    k_merge_cells<IO><<<hs[0], T, smem, st>>>(io, g, ord, list, key, nmax, ctx->dc);
                else
                    k_cap_columns<IO, AT><<<hs[0], T, smem, st>>>(io, g, bA, ord, list, key, nmax);
            }
        }
    }

    // (4) rekey and regroup
    if (n > 0) k_rekey<IO><<<nb(n), T, 0, st>>>(io, g, key, n);
    launch_set_sorted(ctx->dc, n, st);
    ctx->n_bound = n;
    HIP_OK(hipGetLastError());
    return result;
}

rt_status sort_current_ext(rt_ctx ctx);

rt_status do_split_merge(rt_ctx ctx, double alpha, int32_t nmax, int32_t mode, rt_stats *out)
{
    prof_begin(ctx, PC_SPLIT);
    rt_status r;
    // the compaction copies every field by slot: the carried ones first come
    // back from their home slots
    r = materialize_carried(ctx);
    if (r == RT_OK && ctx->precision == RT_FP64) {
        r = split_merge_impl<IO64, double4>(ctx, IO64{ctx->s64[ctx->cur], ctx->bp64.f2, ctx->bp64.Gm},
                                            IO64{ctx->s64[1 - ctx->cur], ctx->bp64.f2, ctx->bp64.Gm}, ctx->bp64.A,
                                            alpha, nmax, mode);
        // the state's wave action from the n and extents the pass wrote
        launch_refresh_w64(ctx->s64[ctx->cur], ctx->n_bound, ctx->stream);
    }
    else if (r == RT_OK)
        r = split_merge_impl<IO32, float4>(ctx, IO32{ctx->s32[ctx->cur], ctx->bp32.f2, ctx->bp32.Gm},
                                           IO32{ctx->s32[1 - ctx->cur], ctx->bp32.f2, ctx->bp32.Gm}, ctx->bp32.A,
                                           alpha, nmax, mode);
    prof_end(ctx);  // profile groups do not nest: the regrouping times as a sort
    rt_status r2 = sort_current_ext(ctx);
    if (r == RT_OK) r = r2;
    if (out && r == RT_OK) r = fill_stats(ctx, out);
    return r;
}

// ---------------------------------------------------------------------------
// Continuous launch from a ghost layer (rt_launch; Section 3c, sources).
// Candidate (column c, direction d, phase-speed bin b) at index
// (c * 4 + d) * n_speeds + b: a flag pass, an exclusive scan for the
// positions of the launched volumes (so their order and ids follow the
// candidates' order), and a write pass into the slots after the compacted
// active set.  The background at the column centre and the launch height is
// read from the double-precision fields in both precisions.
// ---------------------------------------------------------------------------
struct LaunchD {
    double z_launch, dt, t_solstice, F_s, F_w, kh, c_min, c_max, c_center, c_width, sw;
    int n_speeds;
    const double *flux_col;  // device copy, or null
    const double *N2;        // [nz][ny][nx]
    const double *f2;        // [ny]
    const double4 *Gm;       // packed Gamma^2 records, null when Gamma = 0
};

#define LAUNCH_PI 3.14159265358979323846
#define LAUNCH_YEAR (365.25 * 86400.0)

// latitudinal profile of the background source (phi in degrees)
__device__ inline double src_alpha(double phi)
{
    if (phi >= 80.0) return fmin(1.0, fmax(0.0, 1.0 - (phi - 80.0) / 5.0));
    if (phi >= 50.0) return 1.0;
    if (phi >= 20.0) return 0.5 * (1.0 - cos(LAUNCH_PI * (phi - 20.0) / 30.0));
    return 0.0;
}

__device__ inline double col_flux(const Grid &g, const LaunchD &p, int c)
{
    if (p.flux_col) return p.flux_col[c];
    if (g.geometry != RT_SPHERICAL) return 0.0;
    const int j = c / g.nx;
    const double phi = (g.y0 + ((double)j + 0.5) * g.dy) * (180.0 / LAUNCH_PI);
    const double tau = (2.0 * LAUNCH_PI) * (p.t_solstice / LAUNCH_YEAR);
    const double fn = src_alpha(phi) * p.F_s + src_alpha(-phi) * p.F_w;
    const double fs = src_alpha(-phi) * p.F_s + src_alpha(phi) * p.F_w;
    return 0.5 * (fn * (1.0 + cos(tau)) + fs * (1.0 - cos(tau)));
}

// the volume launched by candidate (c, d, b), if any
__device__ inline bool launch_bin(const Grid &g, const LaunchD &p, int c, int d, int b, RayD &r)
{
    const double Fc = col_flux(g, p, c);
    if (!(Fc > 0.0)) return false;
    const int i = c % g.nx, j = c / g.nx;
    const double cb = p.c_min + (((double)b + 0.5) * (p.c_max - p.c_min)) / (double)p.n_speeds;
    const double s = (cb - p.c_center) / p.c_width;
    const double Fb = (0.25 * Fc) * (exp(-(s * s)) / p.sw);
    const double x = g.x0 + ((double)i + 0.5) * g.dx, y = g.y0 + ((double)j + 0.5) * g.dy;
    const d64::Axis ax = d64::axis_x(g, x), ay = d64::axis_y(g, y), az = d64::axis_z(g, p.z_launch);
    auto at = [&](int jj, int ii, int kk) { return p.N2[((int64_t)kk * g.ny + jj) * g.nx + ii]; };
    d64::Cell cl;
    cl.wx = ax.w;
    cl.wy = ay.w;
    cl.wz = az.w;
    const double N2 = d64::lerp3(at(ay.i0, ax.i0, az.i0), at(ay.i0, ax.i1, az.i0), at(ay.i1, ax.i0, az.i0),
                                 at(ay.i1, ax.i1, az.i0), at(ay.i0, ax.i0, az.i1), at(ay.i0, ax.i1, az.i1),
                                 at(ay.i1, ax.i0, az.i1), at(ay.i1, ax.i1, az.i1), cl);
    const double f2 = d64::row_lerp(p.f2, ay);
    const double G2 = d64::gam2(p.Gm, d64::cell_of(g, ax, ay, az));
    const double om = p.kh * cb, om2 = om * om;
    if (!(om2 > f2 && om2 < N2) || !(Fb > 0.0)) return false;
    const double kh = p.kh;
    // m^2 + Gamma^2 from the dispersion relation; evanescent where not above Gamma^2
    const double mm = ((kh * kh) * (N2 - om2)) / (om2 - f2) - G2;
    if (!(mm > 0.0)) return false;
    const double m = -sqrt(mm);
    const double k = d == 0 ? kh : (d == 2 ? -kh : 0.0);
    const double l = d == 1 ? kh : (d == 3 ? -kh : 0.0);
    // vertical group velocity of the dispersion relation (cancellation-free form)
    const double kh2 = k * k + l * l, M2 = m * m + G2, K2 = kh2 + M2;
    const double omd = d64::omega_hat(N2, f2, kh2, M2, K2);
    const double cgz = -(((m * kh2) * (N2 - f2)) / (omd * (K2 * K2)));
    const double Dz = cgz * p.dt;
    const double z = p.z_launch + 0.5 * Dz;
    double A = g.dx * g.dy;
    if (g.geometry == RT_SPHERICAL) {
        const double rr = g.a + p.z_launch;
        A = (((rr * rr) * cos(g.y0 + ((double)j + 0.5) * g.dy)) * g.dx) * g.dy;
    }
    const double W = ((Fb * A) * p.dt) / kh;
    const double dk = 0.1 * kh, dm = 0.1 * fabs(m);
    r.x = x;
    r.y = y;
    r.z = z;
    r.k = k;
    r.l = l;
    r.m = m;
    r.dx = g.dx;
    r.dy = g.dy;
    r.dz = Dz;
    r.px = metric_x(g, y, z, g.dx) * dk;
    r.py = metric_y(g, z, g.dy) * dk;
    r.pz = Dz * dm;
    r.W = W;
    r.n = 0.0;
    return true;
}

__global__ void k_launch_flag(const Grid g, LaunchD p, uint32_t *flag, int64_t M)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int b = (int)(q % p.n_speeds), d = (int)((q / p.n_speeds) % 4), c = (int)(q / (4 * (int64_t)p.n_speeds));
    RayD r;
    flag[q] = launch_bin(g, p, c, d, b, r) ? 1u : 0u;
}

__global__ void k_launch_total(const uint32_t *flag, const uint32_t *offs, int64_t M, int64_t *total)
{
    *total = M > 0 ? (int64_t)offs[M - 1] + (int64_t)flag[M - 1] : 0;
}

template <class IO>
__global__ void k_launch_write(IO io, const Grid g, LaunchD p, const uint32_t *flag, const uint32_t *offs, int64_t M,
                               int64_t n0, int64_t next_id, uint32_t *key)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M || !flag[q]) return;
    const int b = (int)(q % p.n_speeds), d = (int)((q / p.n_speeds) % 4), c = (int)(q / (4 * (int64_t)p.n_speeds));
    RayD r;
    if (!launch_bin(g, p, c, d, b, r)) return;
    r.id = next_id + (int64_t)offs[q];
    const uint32_t slot = (uint32_t)(n0 + (int64_t)offs[q]);
    io.put(g, slot, r, true);
    key[slot] = (uint32_t)c;  // a live key: the slot may hold a stale one (a removal reason or a level key)
}

// launched wave action, one block, fixed order
template <class IO>
__global__ __launch_bounds__(256) void k_launch_sum(IO io, int64_t n0, int64_t cnt, DevCounters *dc)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int64_t q = threadIdx.x; q < cnt; q += 256) v += io.wv((uint32_t)(n0 + q));
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dc->n_launched += cnt;
        dc->launched_W += sh[0];
    }
}

template <class IO>
static rt_status launch_impl(rt_ctx ctx, IO cur_io, IO other_io, LaunchD p, uint32_t *flag, uint32_t *offs,
                             uint32_t *parts, int64_t *n_out)
{
    const Grid &g = ctx->g;
    hipStream_t st = ctx->stream;
    const unsigned T = 256;
    auto nb = [&](int64_t m) { return (unsigned)((m + T - 1) / T > 0 ? (m + T - 1) / T : 1); };
    const int64_t M = (int64_t)g.ncol * 4 * p.n_speeds;
    DevCounters h;
    HIP_OK(hipMemcpyAsync(&h, ctx->dc, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int64_t n = h.n_active;
    k_launch_flag<<<nb(M), T, 0, st>>>(g, p, flag, M);
    HIP_OK(hipMemcpyAsync(offs, flag, sizeof(uint32_t) * (size_t)M, hipMemcpyDeviceToDevice, st));
    scan_u32(offs, M, parts, st);
    k_launch_total<<<1, 1, 0, st>>>(flag, offs, M, &ctx->dc->split_extra);
    int64_t total = 0;
    HIP_OK(hipMemcpyAsync(&total, &ctx->dc->split_extra, sizeof(total), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *n_out = total;
    if (n + total > ctx->cap)
        return rt_fail(ctx, RT_E_CAPACITY, "launch needs %lld ray volumes, capacity %lld", (long long)(n + total),
                       (long long)ctx->cap);
    // compact the active set into the spare buffer in column order, append
    const int nxt = 1 - ctx->cur;
    if (n > 0) k_compact<IO><<<nb(n), T, 0, st>>>(cur_io, other_io, ctx->perm, ctx->skeys, ctx->key[nxt], ctx->dc);
    ctx->cur = nxt;
    uint32_t *key = ctx->key[ctx->cur];
    if (total > 0) {
        k_launch_write<IO><<<nb(M), T, 0, st>>>(other_io, g, p, flag, offs, M, n, h.next_id, key);
        k_launch_sum<IO><<<1, 256, 0, st>>>(other_io, n, total, ctx->dc);
        h.next_id += total;
        HIP_OK(hipMemcpyAsync(&ctx->dc->next_id, &h.next_id, sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    if (n + total > 0) k_rekey<IO><<<nb(n + total), T, 0, st>>>(other_io, g, key, n + total);
    launch_set_sorted(ctx->dc, n + total, st);
    ctx->n_bound = n + total;
    HIP_OK(hipGetLastError());
    return RT_OK;
}

rt_status do_launch(rt_ctx ctx, const rt_launch_params *lp, const double *flux_dev, uint32_t *scratch,
                    int64_t *n_launched)
{
    const Grid &g = ctx->g;
    LaunchD p;
    p.z_launch = lp->z_launch;
    p.dt = lp->dt;
    p.t_solstice = lp->t_solstice;
    p.F_s = lp->F_s;
    p.F_w = lp->F_w;
    p.kh = (2.0 * LAUNCH_PI) / lp->lambda_h;
    p.c_min = lp->c_min;
    p.c_max = lp->c_max;
    p.c_center = lp->c_center;
    p.c_width = lp->c_width;
    p.n_speeds = lp->n_speeds;
    p.flux_col = flux_dev;
    p.N2 = ctx->bg64.N2;
    p.f2 = ctx->bg64.f2;
    p.Gm = ctx->bp64.Gm;
    // spectral weights normalised over the bins, summed in bin order as the
    // definition reads
    double sw = 0.0;
    for (int b = 0; b < lp->n_speeds; b++) {
        const double cb = lp->c_min + (((double)b + 0.5) * (lp->c_max - lp->c_min)) / (double)lp->n_speeds;
        const double s = (cb - lp->c_center) / lp->c_width;
        sw += exp(-(s * s));
    }
    p.sw = sw;
    const int64_t M = (int64_t)g.ncol * 4 * lp->n_speeds;
    uint32_t *flag = scratch, *offs = scratch + M, *parts = offs + M;
    prof_begin(ctx, PC_SPLIT);
    rt_status r;
    // the compaction copies every field by slot: the carried ones first come
    // back from their home slots
    r = materialize_carried(ctx);
    if (r == RT_OK && ctx->precision == RT_FP64) {
        r = launch_impl<IO64>(ctx, IO64{ctx->s64[ctx->cur], ctx->bp64.f2}, IO64{ctx->s64[1 - ctx->cur], ctx->bp64.f2},
                              p, flag, offs, parts, n_launched);
        launch_refresh_w64(ctx->s64[ctx->cur], ctx->n_bound, ctx->stream);
    }
    else if (r == RT_OK)
        r = launch_impl<IO32>(ctx, IO32{ctx->s32[ctx->cur], ctx->bp32.f2}, IO32{ctx->s32[1 - ctx->cur], ctx->bp32.f2},
                              p, flag, offs, parts, n_launched);
    prof_end(ctx);
    if (r != RT_OK) return r;
    return sort_current_ext(ctx);
}

int64_t launch_scratch_len(const Grid &g, int n_speeds)
{
    const int64_t M = (int64_t)g.ncol * 4 * n_speeds;
    return 2 * M + scan_tmp_len(M);
}
