// Per-column flux deposition shared by both precisions.
//
// Ray volumes arrive grouped by column (radix sort on the column key).  A
// workgroup of CPW waves owns CPW consecutive columns, one per wave (CPW = 4,
// or 1 when four columns' profiles would not fit 64 KiB of LDS);
// each wave walks its column's volumes in chunks of 64 in sorted order.
// Within a chunk every contribution is converted to an integer in a
// fixed-point format chosen from the chunk's largest possible contribution
// (below 2^51 units) and added into an int64 profile in the wave's LDS;
// integer addition is associative, so the chunk total does not depend on the
// order in which lanes arrive.  Chunk totals are added to a double profile in
// chunk order.  The result is therefore bitwise reproducible from run to run,
// with no floating-point atomics, and each contribution is rounded once at
// the level of the chunk maximum's last bit -- the accuracy of an ordinary
// double sum.  A chunk whose levels and interfaces lie within eight slots
// (the usual case in a column sorted by level) instead adds its
// contributions in double, level by level, in a fixed order (see the chunk
// loop).  At the end the finished profiles are written together, so that the
// columns of one (field, level) row form one contiguous segment of the
// [NF][nz+1][ncol] output.  The payload decides the fields: P::NL fields
// spread over the levels the volume overlaps (cell means) and P::NI over the
// staggered interface cells (the flux deposition: 4 horizontal and 2
// vertical pseudo-momentum fluxes; the saturation sums: 2 level fields).
#pragma once
#include "rt_internal.h"
#include <type_traits>

// round x * 2^e (|x * 2^e| <= 2^51) to the nearest
// integer, ties to even: adding 1.5 * 2^52 puts the integer part in the low
// mantissa bits of a double whose unit in the last place is 1
__device__ inline long long to_fixed(double x, int e)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = ldexp(x, e) + magic;
    return (long long)(__double_as_longlong(y) - __double_as_longlong(magic));
}

// biased binary exponent of |x| (0 for zero)
__device__ inline int bexp(double x) { return (int)((__double_as_longlong(x) >> 52) & 0x7ff); }

// ordering of this wave's LDS accesses across its lanes
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// sum of v over lane i and lane i + OFF (OFF = 16, 32: exactly lane i xor
// OFF, by the half-row and half-wave swaps of CDNA4) or, within each row of
// 16 lanes, lane (i + OFF) mod 16 (OFF = 2, 4, 8); every form keeps the lane
// index modulo OFF, and the rounding of each lane's sum is fixed by the lane
template <int OFF>
__device__ inline double lane_pair_sum(double v)
{
    if constexpr (OFF >= 16) {
        const uint32_t lo = (uint32_t)__double2loint(v), hi = (uint32_t)__double2hiint(v);
        const auto a = OFF == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                                 : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = OFF == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                                 : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
    } else {
        return v + __builtin_amdgcn_update_dpp(0.0, v, 0x120 + OFF, 0xf, 0xf, false);  // row_ror:OFF
    }
}

// Level window of L levels (and interfaces) k0 .. k0 + L - 1 for a chunk of
// 64 volumes staged at vd (zb, zt, then NF densities, each [64]): lane i takes
// level k0 + s, s = (i - k0) mod L, for the volumes gi, gi + 64/L, ... of the
// chunk (gi = i / L), so that the lane that keeps level k in its registers
// (lane k mod 64) is one of the 64/L lanes summing it; the partial sums of
// those lanes, L apart, are then added by a fixed tree of lane exchanges.
template <class P, int L>
__device__ inline void chunk_window(const Grid &g, const double *vd, int k0, int lane,
                                    double (&preg)[P::NL + P::NI][2])
{
    constexpr int NL = P::NL, NF = P::NL + P::NI, G = 64 / L;
    const int sl = (lane - k0) & (L - 1), gi = lane / L, k = k0 + sl;
    const double lv = (double)k * g.dz, hv = (double)(k + 1) * g.dz;
    double lv2 = ((double)k - 0.5) * g.dz, hv2 = ((double)k + 0.5) * g.dz;
    if (lv2 < 0.0) lv2 = 0.0;
    if (hv2 > g.Lz) hv2 = g.Lz;
    const bool lev_ok = k <= g.nz - 1, itf_ok = k <= g.nz;
    double sm[NF];
#pragma unroll
    for (int q = 0; q < NF; q++) sm[q] = 0.0;
#pragma unroll
    for (int i = 0; i < L; i++) {
        const int j = gi + G * i;
        const double zbj = vd[j], ztj = vd[64 + j];
        double o = fmin(ztj, hv) - fmax(zbj, lv);
        double o2 = fmin(ztj, hv2) - fmax(zbj, lv2);
        o = (lev_ok && o > 0.0) ? o : 0.0;
        o2 = (itf_ok && o2 > 0.0) ? o2 : 0.0;
#pragma unroll
        for (int q = 0; q < NL; q++) sm[q] += vd[128 + 64 * q + j] * o;
#pragma unroll
        for (int q = NL; q < NF; q++) sm[q] += vd[128 + 64 * q + j] * o2;
    }
#pragma unroll
    for (int q = 0; q < NF; q++) {
        if (L <= 2) sm[q] = lane_pair_sum<2>(sm[q]);
        if (L <= 4) sm[q] = lane_pair_sum<4>(sm[q]);
        sm[q] = lane_pair_sum<8>(sm[q]);
        sm[q] = lane_pair_sum<16>(sm[q]);
        sm[q] = lane_pair_sum<32>(sm[q]);
    }
    // level k0 + s (s < L) is kept by lane (k0 + s) mod 64, in register slot
    // (k0 + s) / 64
    const bool take = ((lane - k0) & 63) < L, hi_slot = k >= 64;
#pragma unroll
    for (int q = 0; q < NF; q++) {
        preg[q][0] += (take && !hi_slot) ? sm[q] : 0.0;
        preg[q][1] += (take && hi_slot) ? sm[q] : 0.0;
    }
}

// A payload may split its per-volume work into fetch(slot, raw), the loads,
// and cook(raw, column, zb, zt, bv), the arithmetic, so that the deposition
// can issue a chunk's loads one chunk ahead; any other payload is fetched as
// its slot and cooked by load().
template <class P, class = void>
struct DepSplit {
    using Raw = uint32_t;
    __device__ static void fetch(const P &, uint32_t s, Raw &r) { r = s; }
    __device__ static void cook(const P &p, const Raw &r, int c, double &zb, double &zt, double *bv)
    {
        p.load(r, c, zb, zt, bv);
    }
};
template <class P>
struct DepSplit<P, std::void_t<typename P::Raw>> {
    using Raw = typename P::Raw;
    __device__ static void fetch(const P &p, uint32_t s, Raw &r) { p.fetch(s, r); }
    __device__ static void cook(const P &p, const Raw &r, int c, double &zb, double &zt, double *bv)
    {
        p.cook(r, c, zb, zt, bv);
    }
};

// P::load(slot, column, zb, zt, bv[NF]) fills the vertical span of the volume
// (in the column the sort grouped it in) and its NF densities per unit
// height (for the fluxes: (cgx k, cgx l, cgy k, cgy l, cgz k, cgz l) * W / Dz).
//
// Each wave owns dep_wave_words() 64-bit words of LDS: its integer profile
// [NF][nzp] and, in the register-profile mode, the staging of a chunk for the
// level-parallel path ((2 + NF) x 64 words).
//
// P::WAVES: waves per SIMD the register-profile form is built for (fewer for
// payloads with more fields or more live values, so that nothing spills).
//
// RP: with at most 128 levels and interfaces the double profile of a wave's
// column lives in registers (lane j holds levels j and j + 64 of every
// field), which halves the LDS of a workgroup; at the end it is stored over
// the wave's own integer profile (all zero by then) for the common write-out.
template <class P, bool RP>
__host__ __device__ inline int dep_wave_words(int nzp)
{
    constexpr int NF = P::NL + P::NI;
    return RP ? max(NF * nzp, (2 + NF) * 64) : NF * nzp;
}

template <class P, int CPW, bool RP>
__global__ __launch_bounds__(64 * CPW, RP ? P::WAVES : 2) void k_deposit(Grid g, P pl, const uint32_t *__restrict__ perm,
                                                      const uint32_t *__restrict__ colstart, double *__restrict__ flux)
{
    constexpr int NL = P::NL, NF = P::NL + P::NI;
    static_assert(NF % 2 == 0 && NF <= 16, "fields are reduced in pairs");
    extern __shared__ unsigned long long dep_smem[];
    const int nzp = g.nz + 1;
    const int WR = dep_wave_words<P, RP>(nzp);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    unsigned long long *acc = dep_smem + (size_t)wave * WR;  // this wave's [NF][nzp]
    // [CPW][NF][nzp] finished profiles (stride WR): after the integer ones, or
    // over each wave's own
    double *profs = (double *)(dep_smem + (RP ? 0 : (size_t)CPW * WR));
    double *prof = profs + (size_t)wave * WR;
    double preg[NF][2];
#pragma unroll
    for (int q = 0; q < NF; q++) preg[q][0] = preg[q][1] = 0.0;
    // runs of consecutive workgroups stay on one XCD, so that neighbouring
    // columns share its L2 (the state lines at column boundaries, the flux
    // rows written 32 bytes per workgroup)
    const int c_first = (int)xcd_block(gridDim.x) * CPW;
    const int ncols = min(CPW, g.ncol - c_first);
    for (int e = lane; e < WR; e += 64) {
        acc[e] = 0ull;
        if (!RP) prof[e] = 0.0;
    }
    wave_sync();
    if (wave < ncols) {
        const int c = c_first + wave;
        const uint32_t s0 = colstart[c], s1 = colstart[c + 1];
        // loads run ahead of the arithmetic: the state of the next chunk and
        // the slots of the one after are in flight while a chunk is summed
        using Split = DepSplit<P>;
        typename Split::Raw raw{};
        uint32_t pn = s0 + 64u + (uint32_t)lane < s1 ? perm[s0 + 64u + (uint32_t)lane] : 0u;
        if (s0 + (uint32_t)lane < s1) Split::fetch(pl, perm[s0 + (uint32_t)lane], raw);
        for (uint32_t base = s0; base < s1; base += 64) {
            const uint32_t r = base + (uint32_t)lane;
            const bool valid = r < s1;
            const typename Split::Raw cur = raw;
            if (r + 64u < s1) Split::fetch(pl, pn, raw);
            pn = r + 128u < s1 ? perm[r + 128u] : 0u;
            double zb = 0.0, zt = 0.0, bv[NF];
#pragma unroll
            for (int q = 0; q < NF; q++) bv[q] = 0.0;
            if (valid) Split::cook(pl, cur, c, zb, zt, bv);
            // the levels (lo .. hi) and interfaces (lo2 .. hi2) the volume
            // overlaps, in level units: the double-precision payload divides
            // (so it visits the same levels as a plain division); the
            // single-precision one multiplies by 1/dz, which can differ only
            // where a bound lies within rounding of an interface, and then by
            // an overlap a few units in the last place of z wide
            int lo = 0x7fffffff, hi = -1, lo2 = 0x7fffffff, hi2 = -1;
            if (valid) {
                const double zbl = P::EXACT_LEVELS ? zb / g.dz : zb * pl.inv_dz;
                const double ztl = P::EXACT_LEVELS ? zt / g.dz : zt * pl.inv_dz;
                lo = max((int)floor(zbl), 0);
                hi = min((int)floor(ztl), g.nz - 1);
                if (P::NI > 0) {
                    lo2 = max((int)floor(zbl + 0.5), 0);
                    hi2 = min((int)floor(ztl + 0.5), g.nz);
                }
            }
            const int k0 = wave_min_i(min(lo, lo2)), k1 = wave_max_i(max(hi, hi2));
            if (RP && k1 - k0 < 8) {
                // Chunk within eight levels (a column sorted by level): the
                // chunk is staged in the wave's LDS (its integer profile, zero
                // between chunks) and summed level by level in double, in a
                // fixed order, with no fixed-point scale; the window is the
                // narrowest of 2, 4 or 8 levels that holds the chunk
                double *vd = (double *)acc;
                vd[lane] = zb;
                vd[64 + lane] = zt;
#pragma unroll
                for (int q = 0; q < NF; q++) vd[128 + 64 * q + lane] = bv[q];
                wave_sync();
                if (k1 - k0 < 2)
                    chunk_window<P, 2>(g, vd, k0, lane, preg);
                else if (k1 - k0 < 4)
                    chunk_window<P, 4>(g, vd, k0, lane, preg);
                else
                    chunk_window<P, 8>(g, vd, k0, lane, preg);
                wave_sync();
#pragma unroll
                for (int t = 0; t < 2 + NF; t++) acc[64 * t + lane] = 0ull;
                wave_sync();
                continue;
            }
            const double h = valid ? fmin(zt - zb, g.dz) : 0.0;
            // per field: the largest possible contribution of the chunk sets
            // the fixed-point scale (a bound on each |bv * overlap|)
            int sx[NF];
#pragma unroll
            for (int q = 0; q < NF; q += 2) {
                // two 11-bit exponents per reduction
                const uint32_t pm = wave_max_u16x2(((uint32_t)bexp(fabs(bv[q]) * h) << 16) |
                                                   (uint32_t)bexp(fabs(bv[q + 1]) * h));
                const int ea = (int)(pm >> 16), eb = (int)(pm & 0xffffu);
                sx[q] = (ea > 0 && ea < 0x7fe) ? 51 - (ea - 1022) : 0;
                sx[q + 1] = (eb > 0 && eb < 0x7fe) ? 51 - (eb - 1022) : 0;
            }
            if (valid) {
                // columns sorted by level put the lanes of a chunk on the same
                // levels: each lane starts its level loop at an offset of its
                // own, so that one LDS add instruction spreads over several
                // words instead of serialising on one (integer adds commute,
                // so the sums do not depend on the order)
                const int nk = hi - lo + 1;
                int kk = nk > 0 ? lo + lane % nk : lo;
                for (int t = 0; t < nk; t++, kk = kk == hi ? lo : kk + 1) {
                    const double lv = (double)kk * g.dz, hv = (double)(kk + 1) * g.dz;
                    const double o = fmin(zt, hv) - fmax(zb, lv);
                    if (!(o > 0.0)) continue;
#pragma unroll
                    for (int q = 0; q < NL; q++) {
                        const long long v = to_fixed(bv[q] * o, sx[q]);
                        if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                    }
                }
                if (P::NI > 0) {
                    const int nk2 = hi2 - lo2 + 1;
                    kk = nk2 > 0 ? lo2 + lane % nk2 : lo2;
                    for (int t = 0; t < nk2; t++, kk = kk == hi2 ? lo2 : kk + 1) {
                        double lv = ((double)kk - 0.5) * g.dz, hv = ((double)kk + 0.5) * g.dz;
                        if (lv < 0.0) lv = 0.0;
                        if (hv > g.Lz) hv = g.Lz;
                        const double o = fmin(zt, hv) - fmax(zb, lv);
                        if (!(o > 0.0)) continue;
#pragma unroll
                        for (int q = NL; q < NF; q++) {
                            const long long v = to_fixed(bv[q] * o, sx[q]);
                            if (v) atomicAdd(&acc[q * nzp + kk], (unsigned long long)v);
                        }
                    }
                }
            }
            // move the chunk's integer sums into the double profile, levels
            // the chunk touched only
            wave_sync();
            if (RP) {
#pragma unroll
                for (int sl = 0; sl < 2; sl++) {
                    const int kk = lane + 64 * sl;
                    if (kk >= k0 && kk <= k1) {
#pragma unroll
                        for (int q = 0; q < NF; q++) {
                            const int at = q * nzp + kk;
                            const long long v = (long long)acc[at];
                            if (v) {
                                preg[q][sl] += ldexp((double)v, -sx[q]);
                                acc[at] = 0ull;
                            }
                        }
                    }
                }
            } else if (k1 >= k0) {
                const int span = k1 - k0 + 1;
                for (int e = lane; e < NF * span; e += 64) {
                    const int q = e / span, kk = k0 + e % span;
                    const int at = q * nzp + kk;
                    const long long v = (long long)acc[at];
                    if (v) {
                        int sq = sx[0];
#pragma unroll
                        for (int t = 1; t < NF; t++) sq = q == t ? sx[t] : sq;
                        prof[at] += ldexp((double)v, -sq);
                        acc[at] = 0ull;
                    }
                }
            }
            wave_sync();
        }
    }
    if (RP) {
        wave_sync();
#pragma unroll
        for (int sl = 0; sl < 2; sl++) {
            const int kk = lane + 64 * sl;
            if (kk < nzp) {
#pragma unroll
                for (int q = 0; q < NF; q++) prof[q * nzp + kk] = preg[q][sl];
            }
        }
    }
    __syncthreads();
    // divide by the cell volume (levels) or staggered-cell volume (interfaces);
    // consecutive threads take consecutive columns of one (field, level) row,
    // so a thread keeps one column (64 CPW is a multiple of CPW)
    const int cl = tid % CPW;
    if (cl >= ncols) return;
    const int c = c_first + cl;
    const double area_h = g.dx * g.dy;
    const double cphi = g.geometry == RT_SPHERICAL ? cos(g.y0 + ((double)(c / g.nx) + 0.5) * g.dy) : 1.0;
    for (int e = tid; e < CPW * NF * nzp; e += 64 * CPW) {
        const int qk = e / CPW;
        const int q = qk / nzp, kk = qk % nzp;
        const double acc_v = profs[(size_t)cl * WR + qk];
        double val;
        if (q < NL) {
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

template <class P, int CPW, bool RP>
inline size_t deposit_smem(const Grid &g)
{
    return (size_t)((RP ? 1 : 2) * CPW) * (size_t)dep_wave_words<P, RP>(g.nz + 1) * 8;
}

// launch with four columns per workgroup when their profiles fit 64 KiB of
// LDS, else one; register profiles up to 128 levels and interfaces
template <class P, bool RP>
inline void launch_deposit_rp(const Grid &g, const P &p, const uint32_t *perm, const uint32_t *colstart,
                              double *flux, hipStream_t s)
{
    if (deposit_smem<P, 4, RP>(g) <= 65536)
        k_deposit<P, 4, RP><<<(unsigned)((g.ncol + 3) / 4), 256, deposit_smem<P, 4, RP>(g), s>>>(g, p, perm, colstart,
                                                                                                 flux);
    else
        k_deposit<P, 1, RP><<<(unsigned)g.ncol, 64, deposit_smem<P, 1, RP>(g), s>>>(g, p, perm, colstart, flux);
}

template <class P>
inline void launch_deposit_k(const Grid &g, const P &p, const uint32_t *perm, const uint32_t *colstart, double *flux,
                             hipStream_t s)
{
    if (g.nz + 1 <= 128)
        launch_deposit_rp<P, true>(g, p, perm, colstart, flux, s);
    else
        launch_deposit_rp<P, false>(g, p, perm, colstart, flux, s);
}
