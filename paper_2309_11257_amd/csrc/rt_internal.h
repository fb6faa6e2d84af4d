// Internal declarations of the gfx950 ray-volume tracer library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rt.h"

// Keys of removed ray volumes sort after every column key: ncol + reason.
enum { RK_TOP = 0, RK_BOTTOM = 1, RK_POLE = 2, RK_INVALID = 3, RK_MERGED = 4, RK_CAPPED = 5, RK_NREASON = 6 };

struct Grid {
    int geometry, nx, ny, nz;
    int ncol;
    double dx, dy, dz, x0, y0, a;
    double Lx, Ly, Lz;
    double pole;  // latitude beyond which ray volumes are removed (rad)
};

template <typename T>
struct Bg {
    const T *U, *V, *N2;
    const T *Ux, *Uy, *Uz, *Vx, *Vy, *Vz, *N2x, *N2y, *N2z;
    const T *f2, *f2y;   // [ny]
    const double *rho;   // [nz]
};

// Packed double-precision background for cell (column c, level k) at index
// c*nz + k:  A = (U, V, N2, Ux), G = (Uy, Uz, Vx, Vy), (Vz, N2x, N2y, N2z);
// f^2 and (f^2)_y by latitude row [ny] (their trilinear interpolation of the
// row-replicated field equals the linear one between rows, bit for bit).
// A column's levels are contiguous; a trilinear corner costs one 32-byte load
// per record.
struct Bg64P {
    const double4 *A;  // [ncol*nz]
    const double4 *G;  // [ncol*nz*2]
    const double *f2, *f2y;
    const double4 *Gm;  // [ncol*nz] (Gamma^2, its x, y, z gradients); null when Gamma = 0
};

// Packed single-precision background for cell (column c, level k) at index
// c*nz + k:  A = (U, V, N2, Ux), G = (Uy, Uz, Vx, Vy), (Vz, N2x, N2y, N2z);
// f^2 and (f^2)_y by latitude row [ny].  The step's face evaluations need
// only A; the centre needs A and both G records.
struct Bg32P {
    const float4 *A;  // [ncol*nz]
    const float4 *G;  // [ncol*nz*2]
    const float *f2, *f2y;
    const float4 *Gm;  // [ncol*nz] (Gamma^2, its x, y, z gradients); null when Gamma = 0
};

// double-precision state: absolute coordinates, as the public interface
struct S64 {
    double *x, *y, *z, *k, *l, *m, *dx, *dy, *dz, *px, *py, *pz, *n;
    int64_t *id;
    // the wave action ((n px) py) pz of each slot, carried with the state
    // and refreshed wherever n or an extent changes (load, saturation,
    // split/merge, launch)
    double *W;
    // the fields a step does not change (px, py, pz, n, id) stay where they
    // were when the steps began: hm[slot] is the slot that holds them, or hm
    // is null when they are stored at the slot itself
    uint32_t *hm;
    __host__ __device__ uint32_t home(uint32_t s) const { return hm ? hm[s] : s; }
};

// single-precision state: horizontal position as column index + offset in
// cell units, height as level index + offset in level units; extents Dx, Dy
// in cell units, Dz in metres.  The vertical wavenumber m and the wave
// action W are held in double: m grows without bound towards a critical
// level, and the single-precision rounding of its running sum (at every RK
// stage, and once more when stored) is what single-precision state loses
// most drag accuracy to; every operation on m is still single precision
struct S32 {
    uint32_t *col;
    int32_t *lev;
    float *xi, *eta, *zeta, *k, *l, *dxi, *deta, *dz, *px, *py, *pz;
    double *m;
    double *W;
    int64_t *id;
    // N^2, f^2 and Gamma^2 at the carrier, written by the step that produced
    // the state (the deposition's background; valid while ctx->car_ok)
    float *cn2, *cf2, *cg2;
    // the fields a step does not change (px, py, pz, id) stay where they
    // were when the steps began: hm[slot] is the slot that holds them, or
    // hm is null when they are stored at the slot itself
    uint32_t *hm;
};

// device-side counters (one instance per context)
struct DevCounters {
    int64_t n_sorted;   // keys in the last sort (slots in the current buffer)
    int64_t n_active;   // sorted keys that name a column
    int64_t removed[RK_NREASON];
    double removed_W;
    int64_t n_split, n_merged;
    int64_t split_extra;
    int64_t next_id;
    int64_t steps;
    int64_t n_launched;  // volumes launched (cumulative)
    double launched_W;   // their wave action (cumulative)
    uint64_t bad_key;    // ~id of the smallest id deactivated as non-finite or degenerate since the
                         // last report (the largest complement), 0 if none
};

// Scratch of the regrouping after a step (sort.hip): per-column counters
// (zero between regroupings), offsets, per-tile counts and arrival buckets
struct RegroupBufs {
    uint32_t *inc, *inlow, *outc, *mfill, *mstart, *lpc;  // [ncol]
    uint32_t *cnew;                                       // [ncol + 1]
    uint32_t *tmv;                                        // [tiles] changed keys per tile, then their prefix
    uint32_t *rtc;                                        // [RK_NREASON][tiles] removed per tile, then prefix
    uint32_t *mbuf;                                       // [capacity] arrivals, by destination column
    uint32_t *scratch;                                    // [regroup_scratch_words] (8-byte aligned)
};

struct rt_ctx_s {
    rt_config cfg;
    Grid g;
    hipStream_t stream;
    int device;  // the HIP device current at rt_create
    char err[512];
    int precision;
    // background
    bool have_bg;
    Bg<double> bg64;
    Bg64P bp64;
    Bg32P bp32;
    double *rho;
    double *coslat;  // cos of the row-centre latitudes [ny] (spherical drag)
    // state: double buffers
    S64 s64[2];
    S32 s32[2];
    uint32_t *key[2];
    int cur;
    // hm arrays of the two buffers; while hm_on the current buffer's px,
    // py, pz and id (and n in double precision) are those of buffer `home` at
    // the slots its hm names (rt_step leaves them in place; an operation that
    // rewrites the set first gathers them back, see materialize_carried)
    uint32_t *hm_b[2];
    bool hm_on;
    int home;
    int64_t n_sorts;  // regrouping sorts since the last load (some refine by level)
    int64_t cap;
    int64_t n_bound;  // host-side upper bound of active count (the device holds the exact one)
    bool have_rays;
    bool car_ok;  // single precision: the current buffer's carrier background is that of its state (set by rt_step)
    // sorted view of the current buffer
    uint32_t *perm, *skeys;
    uint32_t *colstart;  // [ncol + 1]
    uint32_t *wcol;      // single-precision step: column of each wave (wave table)
    // sort scratch
    uint32_t *tk, *tv, *hist;
    int64_t hist_len;
    // regrouping after a step: second sorted-key and offset arrays (swapped
    // with skeys / colstart) and scratch
    uint32_t *skeys_b, *colstart_b, *perm_b;
    RegroupBufs rg;
    // flux scratch
    double *flux, *drag;
    // saturation: level sums P and sum P_j K_j^2 [2][nz+1][ncol], kappa [nz][ncol]
    double *satpq, *kappa;
    // signed Coriolis parameter by row (double, and float for an FP32 context)
    double *frow;
    float *frow32;
    // full fluxes and budget (allocated on first use): fields [8 or 4][nz+1][ncol],
    // their smoothed copy, tendencies [3][nz][ncol]
    double *full, *fulls, *fullt;
    double *bud, *buds, *budt;
    // launch scratch (flags, positions, scan parts) and the column flux
    uint32_t *lscr;
    int64_t lscr_len;
    double *lflux;
    // scale-height correction (allocated on first use): the field as given and
    // its packed records; bp64.Gm / bp32.Gm point at the records while it is on
    double *g2raw;
    double4 *gm64;
    float4 *gm32;
    // per-column flags: 1 = the surrogate owns the column this step
    uint8_t *frozen;
    bool have_frozen;
    // counters
    DevCounters *dc;
    double *red;      // reduction scratch
    double *tred;     // removal tally partials [256]
    int64_t *ired;    // integer scratch
    uint32_t *sm;     // split/merge scratch
    // allocation bookkeeping
    void *allocs[96];
    int nallocs;
    // profiling (event pairs by kernel class)
    bool prof_on;
    int prof_class;
    void *prof;  // std::vector of records, owned by api.hip
};

enum { PC_STEP = 0, PC_SORT = 1, PC_DEPOSIT = 2, PC_DRAG = 3, PC_SPLIT = 4, PC_STATS = 5, PC_SAT = 6, PC_N = 8 };
void prof_begin(rt_ctx ctx, int cls);
void prof_end(rt_ctx ctx);

// Wave-wide maximum / minimum by data-parallel-primitive lane moves (no LDS
// round trips): within quads, within rows of 16 (half mirror, mirror), then
// across rows (broadcast of lane 15 and lane 31); lane 63 ends with the
// result, which is read back as a wave-uniform value.  All 64 lanes must be
// active.
#define DPP_QUAD_1032 0xB1
#define DPP_QUAD_2301 0x4E
#define DPP_ROW_HALF_MIRROR 0x141
#define DPP_ROW_MIRROR 0x140
#define DPP_ROW_BCAST15 0x142
#define DPP_ROW_BCAST31 0x143
template <bool MAX>
__device__ inline int wave_reduce_i(int v)
{
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_QUAD_1032, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_QUAD_2301, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_ROW_MIRROR, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_ROW_BCAST15, 0xA, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(v, v, DPP_ROW_BCAST31, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ inline int wave_max_i(int v) { return wave_reduce_i<true>(v); }
// wave-wide maximum of the two 16-bit halves of v, each on its own (packed
// 16-bit integer maximum)
__device__ inline uint32_t wave_max_u16x2(uint32_t v)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    auto op = [](uint32_t a, int b) {
        const u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, (uint32_t)b);
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
    };
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_1032, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_2301, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_MIRROR, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST15, 0xA, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST31, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline int wave_min_i(int v) { return wave_reduce_i<false>(v); }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Remap so that runs of XCD_CHUNK consecutive blocks land on one XCD: the
// waves of a run share background columns in that XCD's L2, while the runs
// are dealt round-robin so that every XCD gets an even share of each part
// of the column-sorted range (the cost of a volume depends on where it is:
// one contiguous eighth per XCD left the slowest XCD half as busy again as
// the mean).  The ragged tail beyond whole rounds keeps the plain order.
#define XCD_CHUNK 16
__device__ inline int64_t xcd_lin(int64_t b, int64_t nb)
{
    const int64_t full = nb / (8 * XCD_CHUNK) * (8 * XCD_CHUNK);
    if (b >= full) return b;
    const int64_t x = b & 7, q = b >> 3;  // XCD, and the block's turn on it
    return (q / XCD_CHUNK) * (8 * XCD_CHUNK) + x * XCD_CHUNK + q % XCD_CHUNK;
}
// the same for the block of a one-dimensional grid of nb blocks
__device__ inline int64_t xcd_block(int64_t nb) { return xcd_lin(blockIdx.x, nb); }

// error helpers
rt_status rt_fail(rt_ctx c, rt_status s, const char *fmt, ...);

#define HIP_OK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return rt_fail(ctx, RT_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// launchers (implemented in the kernel translation units)
void launch_gradients64(const Grid &g, const double *U, const double *V, const double *N2, const double *f,
                        double *out12, double *f2, double *f2y, hipStream_t s);
void launch_round32(const double *in, float *out, int64_t n, hipStream_t s);
void launch_pack64(const Grid &g, const Bg<double> &b, double4 *A, double4 *G, hipStream_t s);
void launch_gamma_pack(const Grid &g, const double *G2, double4 *out64, float4 *out32, hipStream_t s);
void launch_pack32(const Grid &g, const Bg<double> &b, float4 *A, float4 *G, hipStream_t s);

void launch_load64(const Grid &g, const rt_rays &in, int64_t n, S64 dst, uint32_t *key, hipStream_t s);
void launch_load32(const Grid &g, const rt_rays &in, int64_t n, S32 dst, uint32_t *key, hipStream_t s);
void launch_store64(const Grid &g, S64 src, const uint32_t *perm, const DevCounters *dc, rt_rays out,
                    int64_t bound, hipStream_t s);
void launch_store32(const Grid &g, S32 src, const uint32_t *perm, const DevCounters *dc, rt_rays out,
                    int64_t bound, hipStream_t s);

void launch_step64(const Grid &g, const Bg64P &b, S64 src, S64 dst, const uint32_t *perm, uint32_t *key_out,
                   const DevCounters *dc, int64_t bound, double dt, const uint8_t *frozen, const uint32_t *skeys,
                   hipStream_t s);
void launch_step32(const Grid &g, const Bg32P &b, S32 src, S32 dst, const uint32_t *perm, uint32_t *key_out,
                   const uint32_t *colstart, const uint32_t *wcol, int64_t bound, double dt,
                   const uint8_t *frozen, const uint32_t *skeys, hipStream_t s);
int64_t wave_table_len(int64_t cap, int ncol);
void launch_features64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s);
void launch_features32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                       float *X, hipStream_t s);

// stable LSD radix sort of keys[0..*n) with 32-bit payload (identity if vals == NULL)
void radix_sort(const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out, uint32_t *vals_out,
                uint32_t *tk, uint32_t *tv, uint32_t *hist, const int64_t *n_dev, int64_t bound, int nbits,
                hipStream_t s);
int64_t radix_hist_len(int64_t bound);

// The stable sort by column of keys written at the positions of the previous
// regrouping (sk_old, cs_old: its sorted keys and column offsets), for at
// most bound keys (n_dev on the device): perm, sk_new, cs_new (and wcol,
// nullable) as the radix sort and launch_colstart give them; dc->n_active set
void regroup_after_step(const uint32_t *key, const uint32_t *sk_old, const uint32_t *cs_old, const int64_t *n_dev,
                        int64_t bound, int ncol, RegroupBufs rb, uint32_t *perm, uint32_t *sk_new, uint32_t *cs_new,
                        uint32_t *wcol, DevCounters *dc, hipStream_t s);
int64_t regroup_tiles(int64_t bound);
// each column's range of pin, stably sorted by level (lev: single-precision
// stored levels, or z and dz: floor(z / dz) clamped to 0 .. nz), into pout
void regroup_levels(const uint32_t *pin, uint32_t *pout, const uint32_t *colstart, int ncol, const int32_t *lev,
                    const double *z, double dz, int nz, hipStream_t s);
// pout[j] = pin[j] for j in [*cs_end, *n_dev) (the removed volumes)
void copy_removed(const uint32_t *pin, uint32_t *pout, const uint32_t *cs_end, const int64_t *n_dev, hipStream_t s);
int64_t regroup_scratch_words(int64_t cap, int ncol);
// in-place exclusive scan of t[0..len) (parts: scan_tmp_len(len) scratch)
void scan_u32(uint32_t *t, int64_t len, uint32_t *parts, hipStream_t s);
int64_t scan_tmp_len(int64_t len);
// column offsets of the sorted keys; with wcol also the step's wave table
void launch_colstart(const uint32_t *skeys, DevCounters *dc, uint32_t *colstart, uint32_t *wcol, int ncol,
                     hipStream_t s);
void launch_levkey32(const Grid &g, S32 st, uint32_t *key, const DevCounters *dc, int64_t bound, hipStream_t s);
void launch_levkey64(const Grid &g, S64 st, uint32_t *key, const DevCounters *dc, int64_t bound, hipStream_t s);
void launch_colkey(uint32_t *skeys, const DevCounters *dc, uint32_t nl, int64_t bound, hipStream_t s);

void launch_tally64(const Grid &g, S64 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc,
                    double *red, hipStream_t s);
void launch_tally32(const Grid &g, S32 st, const uint32_t *perm, const uint32_t *skeys, DevCounters *dc,
                    double *red, hipStream_t s);
void launch_gather_carried(S32 from, S32 to, const uint32_t *hm, const uint32_t *perm, const int64_t *n_dev,
                           int64_t bound, hipStream_t s);
S32 view32(const rt_ctx_s *ctx, int b);
S64 view64(const rt_ctx_s *ctx, int b);
void launch_refresh_w64(S64 st, int64_t n, hipStream_t s);
rt_status materialize_carried(rt_ctx_s *ctx);
void launch_gather_carried64(S64 from, S64 to, const uint32_t *hm, const uint32_t *perm, const int64_t *n_dev,
                             int64_t bound, hipStream_t s);
void launch_stats64(S64 st, const uint32_t *perm, const DevCounters *dc, double *red, int64_t bound, hipStream_t s);
void launch_stats32(S32 st, const uint32_t *perm, const DevCounters *dc, double *red, int64_t bound, hipStream_t s);

void launch_deposit64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, hipStream_t s);
// car: take N^2, f^2 (and Gamma^2) at the carrier from the state's carrier
// arrays instead of interpolating them
void launch_deposit32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart,
                      double *flux, bool car, hipStream_t s);
void launch_drag(const Grid &g, const double *rho, const double *cosr, const double *flux, double *drag, hipStream_t s);
void launch_coslat(const Grid &g, double *cosr, hipStream_t s);
// full fluxes [8][nz+1][ncol], budget fields [4][nz+1][ncol], smoothing of
// [nslices][ncol] slices, the full tendencies [3][nz][ncol] and the budget
// propagation terms [2][nz][ncol]
void launch_full_fluxes64(const Grid &g, const Bg64P &b, S64 st, const double *frow, const uint32_t *perm,
                          const uint32_t *colstart, const double *rho, double *F, hipStream_t s);
void launch_full_fluxes32(const Grid &g, const Bg32P &b, S32 st, const float *frow, const uint32_t *perm,
                          const uint32_t *colstart, const double *rho, double *F, hipStream_t s);
void launch_budget64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *colstart, double *F,
                     hipStream_t s);
void launch_budget32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *colstart, double *F,
                     hipStream_t s);
void launch_smooth(const Grid &g, const double *in, double *out, int64_t nslices, hipStream_t s);
void launch_full_tend(const Grid &g, const double *cosr, const double *rho, const double *frow, const double *F,
                      double *out, hipStream_t s);
void launch_budget_terms(const Grid &g, const double *cosr, const double *F, double *out, hipStream_t s);
// spectral saturation of the current (sorted) set: level sums, kappa, damping
void launch_saturation64(const Grid &g, const Bg64P &b, S64 st, const uint32_t *perm, const uint32_t *skeys,
                         const uint32_t *colstart, const DevCounters *dc, const double *rho, double dt, double *PQ,
                         double *kappa, int64_t bound, hipStream_t s);
void launch_saturation32(const Grid &g, const Bg32P &b, S32 st, const uint32_t *perm, const uint32_t *skeys,
                         const uint32_t *colstart, const DevCounters *dc, const double *rho, double dt, double *PQ,
                         double *kappa, int64_t bound, hipStream_t s);

void launch_copy_n(const uint32_t *src, uint32_t *dst, const DevCounters *dc, int64_t bound, hipStream_t s);
void launch_set_sorted(DevCounters *dc, int64_t n, hipStream_t s);
void launch_maxid(const int64_t *id, int64_t n, DevCounters *dc, hipStream_t s);
void launch_sorted_from_active(DevCounters *dc, hipStream_t s);

// split / merge / cap
rt_status do_split_merge(rt_ctx ctx, double alpha, int32_t nmax, int32_t mode, rt_stats *out);
// continuous launch: scratch of launch_scratch_len() uint32, flux_dev the
// device copy of the column flux or null
rt_status fill_stats(rt_ctx ctx, rt_stats *out);
rt_status do_launch(rt_ctx ctx, const rt_launch_params *lp, const double *flux_dev, uint32_t *scratch,
                    int64_t *n_launched);
int64_t launch_scratch_len(const Grid &g, int n_speeds);
