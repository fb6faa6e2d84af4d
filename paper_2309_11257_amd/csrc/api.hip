// Host side of the C ABI declared in include/rt.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "rt_internal.h"
#include <utility>

rt_status rt_fail(rt_ctx c, rt_status s, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return s;
}

static void *ctx_alloc(rt_ctx c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (c->nallocs >= (int)(sizeof(c->allocs) / sizeof(c->allocs[0]))) return nullptr;
    if (c->cfg.alloc) {
        p = c->cfg.alloc(bytes, c->cfg.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->allocs[c->nallocs++] = p;
    return p;
}

struct ProfRec {
    int cls;
    hipEvent_t a, b;
};
struct Prof {
    std::vector<ProfRec> recs;
    size_t used = 0;
    double ms[PC_N] = {0};
    int64_t n[PC_N] = {0};
};

static void prof_fold(rt_ctx c)
{
    Prof *p = (Prof *)c->prof;
    if (!p || p->used == 0) return;
    (void)hipEventSynchronize(p->recs[p->used - 1].b);
    for (size_t i = 0; i < p->used; i++) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, p->recs[i].a, p->recs[i].b) == hipSuccess) {
            p->ms[p->recs[i].cls] += t;
            p->n[p->recs[i].cls] += 1;
        }
    }
    p->used = 0;
}

// groups must not nest: each prof_begin is closed by a prof_end before the
// next prof_begin
void prof_begin(rt_ctx c, int cls)
{
    if (!c->prof_on) return;
    Prof *p = (Prof *)c->prof;
    if (p->used == 4096) prof_fold(c);
    if (p->used == p->recs.size()) {
        ProfRec r;
        r.cls = cls;
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
        p->recs.push_back(r);
    }
    p->recs[p->used].cls = cls;
    (void)hipEventRecord(p->recs[p->used].a, c->stream);
    c->prof_class = cls;
}

void prof_end(rt_ctx c)
{
    if (!c->prof_on) return;
    Prof *p = (Prof *)c->prof;
    if (p->used < p->recs.size()) {
        (void)hipEventRecord(p->recs[p->used].b, c->stream);
        p->used++;
    }
}

static void prof_destroy(rt_ctx c)
{
    Prof *p = (Prof *)c->prof;
    if (!p) return;
    for (auto &r : p->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    delete p;
    c->prof = nullptr;
}

extern "C" rt_status rt_profile(rt_ctx ctx, int32_t on)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->prof) ctx->prof = new Prof();
    ctx->prof_on = on != 0;
    return RT_OK;
}

extern "C" rt_status rt_profile_read(rt_ctx ctx, double *ms, int64_t *groups)
{
    if (!ctx || !ms || !groups) return rt_fail(ctx, RT_E_ARG, "ms and groups are required");
    for (int i = 0; i < PC_N; i++) {
        ms[i] = 0.0;
        groups[i] = 0;
    }
    Prof *p = (Prof *)ctx->prof;
    if (!p) return RT_OK;
    prof_fold(ctx);
    for (int i = 0; i < PC_N; i++) {
        ms[i] = p->ms[i];
        groups[i] = p->n[i];
        p->ms[i] = 0.0;
        p->n[i] = 0;
    }
    return RT_OK;
}

static void ctx_release(rt_ctx c)
{
    prof_destroy(c);
    for (int i = 0; i < c->nallocs; i++) {
        if (c->cfg.free)
            c->cfg.free(c->allocs[i], c->cfg.user);
        else if (!c->cfg.alloc)
            (void)hipFree(c->allocs[i]);
    }
    c->nallocs = 0;
}

#define ALLOC(ptr, type, count)                                       \
    do {                                                              \
        ptr = (type *)ctx_alloc(ctx, sizeof(type) * (size_t)(count)); \
        if (!ptr) {                                                   \
            ctx_release(ctx);                                         \
            delete ctx;                                               \
            return RT_E_NOMEM;                                        \
        }                                                             \
    } while (0)

extern "C" rt_status rt_create(const rt_config *cfg, rt_ctx *out)
{
    if (!out) return RT_E_ARG;
    *out = nullptr;
    if (!cfg) return RT_E_ARG;
    if (cfg->geometry != RT_CARTESIAN && cfg->geometry != RT_SPHERICAL) return RT_E_ARG;
    if (cfg->precision != RT_FP64 && cfg->precision != RT_FP32) return RT_E_ARG;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return RT_E_ARG;
    if ((int64_t)cfg->nx * cfg->ny > (int64_t)0x7ffffff0) return RT_E_ARG;
    if ((int64_t)cfg->nx * cfg->ny * cfg->nz > (int64_t)0x7ffffff0) return RT_E_ARG;
    if (cfg->nz > 640) return RT_E_UNSUPPORTED;  // per-column deposition profiles in 64 KiB of LDS
    if (!(cfg->dx > 0 && cfg->dy > 0 && cfg->dz > 0)) return RT_E_ARG;
    if (cfg->geometry == RT_SPHERICAL && !(cfg->a > 0)) return RT_E_ARG;
    if (cfg->capacity < 0 || cfg->capacity > (int64_t)0xffffff00) return RT_E_ARG;
    // cell indices are formed with 24-bit products (fewer than 2^24 columns);
    // single-precision lookups address the packed background with 32-bit byte
    // offsets (2 gradient records of 16 B per cell) and its step reads and
    // writes 4-byte ray fields at 32-bit byte offsets
    if ((int64_t)cfg->nx * cfg->ny >= ((int64_t)1 << 24)) return RT_E_UNSUPPORTED;
    if (cfg->precision == RT_FP32 && ((int64_t)cfg->nx * cfg->ny * cfg->nz * 32 >= ((int64_t)1 << 32) ||
                                      cfg->capacity >= ((int64_t)1 << 30)))
        return RT_E_UNSUPPORTED;
    if ((cfg->alloc == nullptr) != (cfg->free == nullptr)) return RT_E_ARG;

    rt_ctx ctx = new rt_ctx_s();
    memset(ctx, 0, sizeof(*ctx));
    ctx->cfg = *cfg;
    ctx->stream = (hipStream_t)cfg->stream;
    ctx->precision = cfg->precision;
    Grid &g = ctx->g;
    g.geometry = cfg->geometry;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.ncol = cfg->nx * cfg->ny;
    g.dx = cfg->dx;
    g.dy = cfg->dy;
    g.dz = cfg->dz;
    g.x0 = 0.0;
    g.y0 = cfg->geometry == RT_SPHERICAL ? -0.5 * M_PI : 0.0;
    g.a = cfg->a;
    g.Lx = (double)g.nx * g.dx;
    g.Ly = (double)g.ny * g.dy;
    g.Lz = (double)g.nz * g.dz;
    g.pole = 89.5 * (3.14159265358979323846 / 180.0);
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return RT_E_DEVICE;
    }

    const int64_t cells = (int64_t)g.ncol * g.nz;
    const int64_t cap = cfg->capacity > 0 ? cfg->capacity : 1;
    ctx->cap = cfg->capacity;

    // background (double always; single copies for an FP32 context)
    double *bgd;
    ALLOC(bgd, double, 12 * cells + 2 * (int64_t)g.ny + g.nz);
    Bg<double> &b = ctx->bg64;
    b.U = bgd;
    b.V = bgd + cells;
    b.N2 = bgd + 2 * cells;
    b.Ux = bgd + 3 * cells;
    b.Uy = bgd + 4 * cells;
    b.Uz = bgd + 5 * cells;
    b.Vx = bgd + 6 * cells;
    b.Vy = bgd + 7 * cells;
    b.Vz = bgd + 8 * cells;
    b.N2x = bgd + 9 * cells;
    b.N2y = bgd + 10 * cells;
    b.N2z = bgd + 11 * cells;
    b.f2 = bgd + 12 * cells;
    b.f2y = bgd + 12 * cells + g.ny;
    ctx->rho = bgd + 12 * cells + 2 * g.ny;
    b.rho = ctx->rho;
    if (ctx->precision == RT_FP64) {
        double4 *pa;
        ALLOC(pa, double4, 3 * cells);
        ctx->bp64.A = pa;
        ctx->bp64.G = pa + cells;
        ctx->bp64.f2 = b.f2;
        ctx->bp64.f2y = b.f2y;
    } else {
        float4 *pa;
        ALLOC(pa, float4, 3 * cells);
        ctx->bp32.A = pa;
        ctx->bp32.G = pa + cells;
    }
    if (ctx->precision == RT_FP32) {
        // single-precision f2 and (f2)_y rows (the fields are rounded into the
        // packed records themselves)
        float *rows;
        ALLOC(rows, float, 2 * (int64_t)g.ny);
        ctx->bp32.f2 = rows;
        ctx->bp32.f2y = rows + g.ny;
        ALLOC(ctx->frow32, float, g.ny);
    }
    ALLOC(ctx->frow, double, g.ny);
    // ray state, two buffers
    for (int buf = 0; buf < 2; buf++) {
        if (ctx->precision == RT_FP64) {
            double *m;
            ALLOC(m, double, 13 * cap);
            S64 &s = ctx->s64[buf];
            double **f[13] = {&s.x, &s.y, &s.z, &s.k, &s.l, &s.m, &s.dx, &s.dy, &s.dz, &s.px, &s.py, &s.pz, &s.n};
            for (int q = 0; q < 13; q++) *f[q] = m + q * cap;
            ALLOC(s.id, int64_t, cap);
            ALLOC(s.W, double, cap);
            ALLOC(ctx->hm_b[buf], uint32_t, cap);
            s.hm = nullptr;
        } else {
            float *m;
            ALLOC(m, float, 11 * cap);
            S32 &s = ctx->s32[buf];
            float **f[11] = {&s.xi, &s.eta, &s.zeta, &s.k, &s.l, &s.dxi, &s.deta, &s.dz, &s.px, &s.py, &s.pz};
            for (int q = 0; q < 11; q++) *f[q] = m + q * cap;
            ALLOC(s.m, double, cap);
            ALLOC(s.col, uint32_t, cap);
            ALLOC(s.lev, int32_t, cap);
            ALLOC(s.W, double, cap);
            ALLOC(s.id, int64_t, cap);
            float *c;
            ALLOC(c, float, 3 * cap);
            s.cn2 = c;
            s.cf2 = c + cap;
            s.cg2 = c + 2 * cap;
            ALLOC(ctx->hm_b[buf], uint32_t, cap);
            s.hm = nullptr;
        }
        ALLOC(ctx->key[buf], uint32_t, cap);
    }
    ALLOC(ctx->perm, uint32_t, cap);
    ALLOC(ctx->skeys, uint32_t, cap);
    ALLOC(ctx->tk, uint32_t, cap);
    ALLOC(ctx->tv, uint32_t, cap);
    ctx->hist_len = radix_hist_len(cap);
    ALLOC(ctx->hist, uint32_t, ctx->hist_len);
    ALLOC(ctx->colstart, uint32_t, (int64_t)g.ncol + 1);
    ALLOC(ctx->colstart_b, uint32_t, (int64_t)g.ncol + 1);
    ALLOC(ctx->skeys_b, uint32_t, cap);
    ALLOC(ctx->perm_b, uint32_t, cap);
    {
        const int64_t nt = regroup_tiles(cap);
        uint32_t *r;
        ALLOC(r, uint32_t, 7 * (int64_t)g.ncol + 1 + (1 + RK_NREASON) * nt);
        RegroupBufs &rb = ctx->rg;
        rb.inc = r;
        rb.inlow = r + g.ncol;
        rb.outc = r + 2 * (int64_t)g.ncol;
        rb.mfill = r + 3 * (int64_t)g.ncol;
        rb.mstart = r + 4 * (int64_t)g.ncol;
        rb.lpc = r + 5 * (int64_t)g.ncol;
        rb.cnew = r + 6 * (int64_t)g.ncol;
        rb.tmv = rb.cnew + g.ncol + 1;
        rb.rtc = rb.tmv + nt;
        ALLOC(rb.mbuf, uint32_t, cap);
        ALLOC(rb.scratch, uint32_t, regroup_scratch_words(cap, g.ncol));
    }
    if (cfg->precision == RT_FP32) ALLOC(ctx->wcol, uint32_t, wave_table_len(cap, g.ncol));
    ALLOC(ctx->flux, double, (int64_t)6 * (g.nz + 1) * g.ncol);
    ALLOC(ctx->drag, double, 2 * cells);
    ALLOC(ctx->satpq, double, (int64_t)2 * (g.nz + 1) * g.ncol);
    ALLOC(ctx->kappa, double, cells);
    ALLOC(ctx->frozen, uint8_t, g.ncol);
    ALLOC(ctx->coslat, double, g.ny);
    ALLOC(ctx->dc, DevCounters, 1);
    ALLOC(ctx->red, double, 8 + 4 * (cap / 256 + 2));
    ALLOC(ctx->tred, double, 256);  // removal tally partials
    ALLOC(ctx->ired, int64_t, 8 + 2 * cap);
    ALLOC(ctx->sm, uint32_t, 8 * cap + 16 + scan_tmp_len(cap));
    if (hipMemsetAsync(ctx->dc, 0, sizeof(DevCounters), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->colstart, 0, sizeof(uint32_t) * ((size_t)g.ncol + 1), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->rg.inc, 0, sizeof(uint32_t) * 4 * (size_t)g.ncol, ctx->stream) != hipSuccess) {
        ctx_release(ctx);
        delete ctx;
        return RT_E_DEVICE;
    }
    launch_coslat(g, ctx->coslat, ctx->stream);
    if (hipGetLastError() != hipSuccess) {
        ctx_release(ctx);
        delete ctx;
        return RT_E_DEVICE;
    }
    ctx->cur = 0;
    ctx->hm_on = false;
    ctx->home = 0;
    *out = ctx;
    return RT_OK;
}

extern "C" rt_status rt_destroy(rt_ctx ctx)
{
    if (!ctx) return RT_E_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    ctx_release(ctx);
    delete ctx;
    return RT_OK;
}

extern "C" const char *rt_last_error(rt_ctx ctx) { return ctx ? ctx->err : "null context"; }

static int bits_of(uint64_t maxkey)
{
    int b = 0;
    while ((1ull << b) <= maxkey) b++;
    return b;
}

// every this many regrouping sorts (and the first after a load) the column
// key is refined by the level
#define LEVEL_REFINE_EVERY 4

// The single-precision state of buffer b as kernels see it: while a run of
// steps leaves px, py, pz and id at their home slots, they are those of the
// home buffer, read through b's hm, and the column of each active volume is
// its key (the step writes no separate column word).
S32 view32(const rt_ctx_s *ctx, int b)
{
    S32 v = ctx->s32[b];
    if (ctx->hm_on) {
        v.col = ctx->key[b];
        const S32 &h = ctx->s32[ctx->home];
        v.px = h.px;
        v.py = h.py;
        v.pz = h.pz;
        v.id = h.id;
        v.hm = ctx->hm_b[b];
    } else {
        v.hm = nullptr;
    }
    return v;
}

// The double-precision state of buffer b as kernels see it: while a run of
// steps leaves px, py, pz, n and id at their home slots, they are those of
// the home buffer, read through b's hm.
S64 view64(const rt_ctx_s *ctx, int b)
{
    S64 v = ctx->s64[b];
    if (ctx->hm_on) {
        const S64 &h = ctx->s64[ctx->home];
        v.px = h.px;
        v.py = h.py;
        v.pz = h.pz;
        v.n = h.n;
        v.id = h.id;
        v.hm = ctx->hm_b[b];
    } else {
        v.hm = nullptr;
    }
    return v;
}

// Gathers the carried fields back to the current buffer's slots (and, in
// single precision, copies the active volumes' columns from their keys)
// before an operation that rewrites the state or adds volumes; afterwards the
// current buffer holds them itself.
rt_status materialize_carried(rt_ctx_s *ctx)
{
    if (!ctx->hm_on) return RT_OK;
    const int cur = ctx->cur, h = ctx->home, t = 1 - h;
    if (ctx->precision == RT_FP32) {
        if (ctx->n_bound > 0)
            HIP_OK(hipMemcpyAsync(ctx->s32[cur].col, ctx->key[cur], sizeof(uint32_t) * (size_t)ctx->n_bound,
                                  hipMemcpyDeviceToDevice, ctx->stream));
        launch_gather_carried(ctx->s32[h], ctx->s32[t], ctx->hm_b[cur], ctx->perm, &ctx->dc->n_sorted, ctx->n_bound,
                              ctx->stream);
        if (t != cur) {
            // the gathered arrays become the current buffer's
            std::swap(ctx->s32[0].px, ctx->s32[1].px);
            std::swap(ctx->s32[0].py, ctx->s32[1].py);
            std::swap(ctx->s32[0].pz, ctx->s32[1].pz);
            std::swap(ctx->s32[0].id, ctx->s32[1].id);
        }
    } else {
        launch_gather_carried64(ctx->s64[h], ctx->s64[t], ctx->hm_b[cur], ctx->perm, &ctx->dc->n_sorted,
                                ctx->n_bound, ctx->stream);
        if (t != cur) {
            std::swap(ctx->s64[0].px, ctx->s64[1].px);
            std::swap(ctx->s64[0].py, ctx->s64[1].py);
            std::swap(ctx->s64[0].pz, ctx->s64[1].pz);
            std::swap(ctx->s64[0].n, ctx->s64[1].n);
            std::swap(ctx->s64[0].id, ctx->s64[1].id);
        }
    }
    ctx->hm_on = false;
    ctx->home = cur;
    HIP_OK(hipGetLastError());
    return RT_OK;
}

// sort the current buffer's keys -> skeys/perm, column offsets, removal
// tallies.  A refining sort orders each column's volumes by level (sort key
// column x (nz + 1) + level, where that fits 32 bits; the sorted keys are
// turned back into column keys); the column sorts in between are stable, so
// the level order persists except for volumes that moved.  The step's waves
// then span few levels and share one stencil box.
//
// after_step: the keys were written by the step at the positions of the
// previous regrouping, whose sorted keys and offsets are still current; a
// column sort is then the regrouping that moves only the volumes that
// changed column (the same permutation as the radix sort)
static rt_status sort_current(rt_ctx ctx, bool after_step = false)
{
    const int64_t bound = ctx->n_bound;
    const uint64_t nl = (uint64_t)ctx->g.nz + 1;
    const uint64_t maxcol = (uint64_t)ctx->g.ncol + RK_NREASON;
    const bool bylev = maxcol * nl <= 0xffffffffull &&
                       ctx->n_sorts % LEVEL_REFINE_EVERY == 0;
    ctx->n_sorts++;
    prof_begin(ctx, PC_SORT);
    if (after_step) {
        // a refining sort: the regrouping, then each column by level (ties
        // keep the regrouping's position order, as in the radix sort of the
        // level-refined key)
        regroup_after_step(ctx->key[ctx->cur], ctx->skeys, ctx->colstart, &ctx->dc->n_sorted, bound, ctx->g.ncol,
                           ctx->rg, bylev ? ctx->perm_b : ctx->perm, ctx->skeys_b, ctx->colstart_b, ctx->wcol,
                           ctx->dc, ctx->stream);
        std::swap(ctx->skeys, ctx->skeys_b);
        std::swap(ctx->colstart, ctx->colstart_b);
        if (bylev) {
            const bool f64 = ctx->precision == RT_FP64;
            regroup_levels(ctx->perm_b, ctx->perm, ctx->colstart, ctx->g.ncol, f64 ? nullptr : ctx->s32[ctx->cur].lev,
                           f64 ? ctx->s64[ctx->cur].z : nullptr, ctx->g.dz, ctx->g.nz, ctx->stream);
            copy_removed(ctx->perm_b, ctx->perm, ctx->colstart + ctx->g.ncol, &ctx->dc->n_sorted, ctx->stream);
        }
        if (ctx->precision == RT_FP64)
            launch_tally64(ctx->g, view64(ctx, ctx->cur), ctx->perm, ctx->skeys, ctx->dc, ctx->tred, ctx->stream);
        else
            launch_tally32(ctx->g, view32(ctx, ctx->cur), ctx->perm, ctx->skeys, ctx->dc, ctx->tred, ctx->stream);
        prof_end(ctx);
        HIP_OK(hipGetLastError());
        return RT_OK;
    }
    if (bylev) {
        if (ctx->precision == RT_FP64)
            launch_levkey64(ctx->g, ctx->s64[ctx->cur], ctx->key[ctx->cur], ctx->dc, bound, ctx->stream);
        else
            launch_levkey32(ctx->g, ctx->s32[ctx->cur], ctx->key[ctx->cur], ctx->dc, bound, ctx->stream);
    }
    radix_sort(ctx->key[ctx->cur], nullptr, ctx->skeys, ctx->perm, ctx->tk, ctx->tv, ctx->hist, &ctx->dc->n_sorted,
               bound, bits_of(bylev ? maxcol * nl - 1 : maxcol), ctx->stream);
    if (bylev) launch_colkey(ctx->skeys, ctx->dc, (uint32_t)nl, bound, ctx->stream);
    launch_colstart(ctx->skeys, ctx->dc, ctx->colstart, ctx->wcol, ctx->g.ncol, ctx->stream);
    if (ctx->precision == RT_FP64)
        launch_tally64(ctx->g, view64(ctx, ctx->cur), ctx->perm, ctx->skeys, ctx->dc, ctx->tred, ctx->stream);
    else
        launch_tally32(ctx->g, view32(ctx, ctx->cur), ctx->perm, ctx->skeys, ctx->dc, ctx->tred, ctx->stream);
    prof_end(ctx);
    HIP_OK(hipGetLastError());
    return RT_OK;
}

rt_status sort_current_ext(rt_ctx ctx) { return sort_current(ctx); }

extern "C" rt_status rt_init_background(rt_ctx ctx, const double *U, const double *V, const double *N2, const double *f,
                                        const double *rho, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!U || !V || !N2 || !rho) return rt_fail(ctx, RT_E_ARG, "U, V, N2 and rho are required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    const int64_t cells = (int64_t)g.ncol * g.nz;
    if (where == RT_HOST) {
        for (int64_t i = 0; i < cells; i++)
            if (!(N2[i] > 0.0) || !std::isfinite(N2[i]) || !std::isfinite(U[i]) || !std::isfinite(V[i]))
                return rt_fail(ctx, RT_E_ARG, "background cell %lld: N2 must be positive and fields finite",
                               (long long)i);
        for (int k = 0; k < g.nz; k++)
            if (!(rho[k] > 0.0)) return rt_fail(ctx, RT_E_ARG, "rho[%d] must be positive", k);
    }
    const hipMemcpyKind kind = where == RT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    double *bgd = (double *)ctx->bg64.U;
    HIP_OK(hipMemcpyAsync(bgd, U, sizeof(double) * cells, kind, ctx->stream));
    HIP_OK(hipMemcpyAsync(bgd + cells, V, sizeof(double) * cells, kind, ctx->stream));
    HIP_OK(hipMemcpyAsync(bgd + 2 * cells, N2, sizeof(double) * cells, kind, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->rho, rho, sizeof(double) * g.nz, kind, ctx->stream));
    // the signed Coriolis parameter by row (zero without f); f^2 and (f^2)_y follow
    if (f)
        HIP_OK(hipMemcpyAsync(ctx->frow, f, sizeof(double) * g.ny, kind, ctx->stream));
    else
        HIP_OK(hipMemsetAsync(ctx->frow, 0, sizeof(double) * g.ny, ctx->stream));
    launch_gradients64(g, ctx->bg64.U, ctx->bg64.V, ctx->bg64.N2, ctx->frow, bgd + 3 * cells, (double *)ctx->bg64.f2,
                       (double *)ctx->bg64.f2y, ctx->stream);
    if (ctx->precision == RT_FP32) {
        launch_round32(bgd + 12 * cells, (float *)ctx->bp32.f2, 2 * (int64_t)g.ny, ctx->stream);
        launch_round32(ctx->frow, ctx->frow32, g.ny, ctx->stream);
        launch_pack32(g, ctx->bg64, (float4 *)ctx->bp32.A, (float4 *)ctx->bp32.G, ctx->stream);
    } else {
        launch_pack64(g, ctx->bg64, (double4 *)ctx->bp64.A, (double4 *)ctx->bp64.G, ctx->stream);
    }
    HIP_OK(hipGetLastError());
    if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->have_bg = true;
    ctx->car_ok = false;  // the carrier background is that of the old fields
    return RT_OK;
}

static rt_status check_rays(rt_ctx ctx, const rt_rays *r)
{
    if (!r || !r->x || !r->y || !r->z || !r->k || !r->l || !r->m || !r->dx || !r->dy || !r->dz || !r->px || !r->py ||
        !r->pz || !r->n || !r->id)
        return rt_fail(ctx, RT_E_ARG, "all ray arrays are required");
    return RT_OK;
}

// device staging for host ray arrays (allocated on first use)
static rt_status stage_rays(rt_ctx ctx, rt_rays *dev, int64_t n)
{
    static const int nf = 13;
    double *m = (double *)ctx_alloc(ctx, sizeof(double) * (size_t)(nf * (n > 0 ? n : 1)) + sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!m) return rt_fail(ctx, RT_E_NOMEM, "staging allocation failed");
    double **f[13] = {&dev->x, &dev->y, &dev->z, &dev->k, &dev->l, &dev->m, &dev->dx, &dev->dy, &dev->dz,
                      &dev->px, &dev->py, &dev->pz, &dev->n};
    for (int q = 0; q < nf; q++) *f[q] = m + (int64_t)q * (n > 0 ? n : 1);
    dev->id = (int64_t *)(m + (int64_t)nf * (n > 0 ? n : 1));
    return RT_OK;
}

static void unstage(rt_ctx ctx, void *p)
{
    // release the most recent staging allocation
    if (ctx->nallocs > 0 && ctx->allocs[ctx->nallocs - 1] == p) {
        ctx->nallocs--;
        if (ctx->cfg.free)
            ctx->cfg.free(p, ctx->cfg.user);
        else if (!ctx->cfg.alloc)
            (void)hipFree(p);
    }
}

extern "C" rt_status rt_set_scale_height(rt_ctx ctx, const double *G2, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!G2) {
        ctx->bp64.Gm = nullptr;
        ctx->bp32.Gm = nullptr;
        ctx->car_ok = false;
        return RT_OK;
    }
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    const int64_t cells = (int64_t)g.ncol * g.nz;
    if (where == RT_HOST)
        for (int64_t i = 0; i < cells; i++)
            if (!(G2[i] >= 0.0) || !std::isfinite(G2[i]))
                return rt_fail(ctx, RT_E_ARG, "Gamma^2 at cell %lld must be finite and non-negative", (long long)i);
    if (!ctx->g2raw) {
        double *raw = (double *)ctx_alloc(ctx, sizeof(double) * (size_t)cells);
        double4 *p64 = (double4 *)ctx_alloc(ctx, sizeof(double4) * (size_t)cells);
        float4 *p32 = ctx->precision == RT_FP32 ? (float4 *)ctx_alloc(ctx, sizeof(float4) * (size_t)cells) : nullptr;
        if (!raw || !p64 || (ctx->precision == RT_FP32 && !p32))
            return rt_fail(ctx, RT_E_NOMEM, "no device memory for the scale-height correction");
        ctx->g2raw = raw;
        ctx->gm64 = p64;
        ctx->gm32 = p32;
    }
    HIP_OK(hipMemcpyAsync(ctx->g2raw, G2, sizeof(double) * (size_t)cells,
                          where == RT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, ctx->stream));
    launch_gamma_pack(g, ctx->g2raw, ctx->gm64, ctx->gm32, ctx->stream);
    HIP_OK(hipGetLastError());
    if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->bp64.Gm = ctx->gm64;
    ctx->bp32.Gm = ctx->gm32;
    ctx->car_ok = false;
    return RT_OK;
}

extern "C" rt_status rt_set_rays(rt_ctx ctx, const rt_rays *rays, int64_t n, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (n < 0) return rt_fail(ctx, RT_E_ARG, "negative ray count");
    if (n > ctx->cap) return rt_fail(ctx, RT_E_CAPACITY, "%lld ray volumes exceed capacity %lld", (long long)n,
                                     (long long)ctx->cap);
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    if (n > 0) {
        rt_status st = check_rays(ctx, rays);
        if (st) return st;
    }
    rt_rays src = {};
    void *staged = nullptr;
    if (n > 0) {
        if (where == RT_HOST) {
            rt_status st = stage_rays(ctx, &src, n);
            if (st) return st;
            staged = src.x;
            const double *hs[13] = {rays->x, rays->y, rays->z, rays->k, rays->l, rays->m, rays->dx,
                                    rays->dy, rays->dz, rays->px, rays->py, rays->pz, rays->n};
            double *ds[13] = {src.x, src.y, src.z, src.k, src.l, src.m, src.dx, src.dy, src.dz, src.px, src.py, src.pz, src.n};
            for (int q = 0; q < 13; q++)
                HIP_OK(hipMemcpyAsync(ds[q], hs[q], sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
            HIP_OK(hipMemcpyAsync(src.id, rays->id, sizeof(int64_t) * n, hipMemcpyHostToDevice, ctx->stream));
        } else {
            src = *rays;
        }
    }
    HIP_OK(hipMemsetAsync(ctx->dc, 0, sizeof(DevCounters), ctx->stream));
    ctx->cur = 0;
    ctx->hm_on = false;
    ctx->home = 0;
    if (ctx->precision == RT_FP64)
        launch_load64(ctx->g, src, n, ctx->s64[0], ctx->key[0], ctx->stream);
    else
        launch_load32(ctx->g, src, n, ctx->s32[0], ctx->key[0], ctx->stream);
    launch_set_sorted(ctx->dc, n, ctx->stream);
    launch_maxid(src.id, n, ctx->dc, ctx->stream);
    ctx->n_bound = n;
    ctx->n_sorts = 0;
    rt_status st = sort_current(ctx);
    if (st) return st;
    if (staged) {
        HIP_OK(hipStreamSynchronize(ctx->stream));
        unstage(ctx, staged);
    }
    ctx->have_rays = true;
    ctx->car_ok = false;  // loaded volumes carry no carrier background
    return RT_OK;
}

extern "C" rt_status rt_step(rt_ctx ctx, double dt, int32_t flags)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg) return rt_fail(ctx, RT_E_STATE, "rt_init_background has not been called");
    if (!ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "rt_set_rays has not been called");
    if (!std::isfinite(dt)) return rt_fail(ctx, RT_E_ARG, "dt must be finite");
    if (flags & ~(RT_STEP_DEPOSIT | RT_STEP_SURROGATE | RT_STEP_SATURATE))
        return rt_fail(ctx, RT_E_ARG, "unknown rt_step flags");
    if ((flags & RT_STEP_SATURATE) && !(dt > 0.0)) return rt_fail(ctx, RT_E_ARG, "saturation needs dt > 0");
    if ((flags & RT_STEP_SURROGATE) && !ctx->have_frozen)
        return rt_fail(ctx, RT_E_STATE, "RT_STEP_SURROGATE needs rt_set_frozen_columns first");
    const uint8_t *frozen = (flags & RT_STEP_SURROGATE) ? ctx->frozen : nullptr;
    const int nxt = 1 - ctx->cur;
    prof_begin(ctx, PC_STEP);
    // the fields a step does not change stay where they are; the step passes
    // on their slots
    if (ctx->precision == RT_FP64) {
        S64 dst = ctx->s64[nxt];
        dst.hm = ctx->hm_b[nxt];
        launch_step64(ctx->g, ctx->bp64, view64(ctx, ctx->cur), dst, ctx->perm, ctx->key[nxt], ctx->dc,
                      ctx->n_bound, dt, frozen, ctx->skeys, ctx->stream);
    } else {
        S32 dst = ctx->s32[nxt];
        dst.hm = ctx->hm_b[nxt];
        launch_step32(ctx->g, ctx->bp32, view32(ctx, ctx->cur), dst, ctx->perm, ctx->key[nxt], ctx->colstart,
                      ctx->wcol, ctx->n_bound, dt, frozen, ctx->skeys, ctx->stream);
    }
    if (!ctx->hm_on) {
        ctx->home = ctx->cur;
        ctx->hm_on = true;
    }
    prof_end(ctx);
    launch_sorted_from_active(ctx->dc, ctx->stream);
    ctx->cur = nxt;
    // the single-precision step wrote the carrier background of the state it produced
    ctx->car_ok = ctx->precision == RT_FP32;
    rt_status st = sort_current(ctx, true);
    if (st) return st;
    if (flags & RT_STEP_SATURATE) {
        st = rt_saturate(ctx, dt, nullptr, RT_DEVICE);
        if (st) return st;
    }
    if (flags & RT_STEP_DEPOSIT) return rt_deposit_flux(ctx, nullptr, nullptr, RT_DEVICE);
    return RT_OK;
}

extern "C" rt_status rt_saturate(rt_ctx ctx, double dt, double *kappa, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (!(dt > 0.0) || !std::isfinite(dt)) return rt_fail(ctx, RT_E_ARG, "dt must be positive and finite");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    prof_begin(ctx, PC_SAT);
    if (ctx->precision == RT_FP64)
        launch_saturation64(g, ctx->bp64, view64(ctx, ctx->cur), ctx->perm, ctx->skeys, ctx->colstart, ctx->dc, ctx->rho,
                            dt, ctx->satpq, ctx->kappa, ctx->n_bound, ctx->stream);
    else
        launch_saturation32(g, ctx->bp32, ctx->s32[ctx->cur], ctx->perm, ctx->skeys, ctx->colstart, ctx->dc, ctx->rho,
                            dt, ctx->satpq, ctx->kappa, ctx->n_bound, ctx->stream);
    prof_end(ctx);
    HIP_OK(hipGetLastError());
    if (kappa) {
        const size_t n = (size_t)g.nz * g.ncol;
        HIP_OK(hipMemcpyAsync(kappa, ctx->kappa, sizeof(double) * n,
                              where == RT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, ctx->stream));
        if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return RT_OK;
}

extern "C" rt_status rt_features(rt_ctx ctx, float *X, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!X) return rt_fail(ctx, RT_E_ARG, "X is required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    const Grid &g = ctx->g;
    const size_t n = (size_t)g.ncol * (size_t)(3 * g.nz + 48);
    float *dst = X;
    void *staged = nullptr;
    if (where == RT_HOST) {
        staged = ctx_alloc(ctx, sizeof(float) * n);
        if (!staged) return rt_fail(ctx, RT_E_NOMEM, "no device memory for the feature matrix");
        dst = (float *)staged;
    }
    if (ctx->precision == RT_FP64)
        launch_features64(g, ctx->bp64, view64(ctx, ctx->cur), ctx->perm, ctx->colstart, dst, ctx->stream);
    else
        launch_features32(g, ctx->bp32, view32(ctx, ctx->cur), ctx->perm, ctx->colstart, dst, ctx->stream);
    HIP_OK(hipGetLastError());
    if (staged) {
        HIP_OK(hipMemcpyAsync(X, dst, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        unstage(ctx, staged);
    }
    return RT_OK;
}

extern "C" rt_status rt_set_frozen_columns(rt_ctx ctx, const uint8_t *mask, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const size_t n = (size_t)ctx->g.ncol;
    if (!mask) {
        HIP_OK(hipMemsetAsync(ctx->frozen, 0, n, ctx->stream));
    } else {
        HIP_OK(hipMemcpyAsync(ctx->frozen, mask, n, where == RT_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                              ctx->stream));
        if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    ctx->have_frozen = true;
    return RT_OK;
}

extern "C" rt_status rt_deposit_flux(rt_ctx ctx, double *flux, double *drag, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    double *fdst = (where == RT_DEVICE && flux) ? flux : ctx->flux;
    double *ddst = (where == RT_DEVICE && drag) ? drag : ctx->drag;
    prof_begin(ctx, PC_DEPOSIT);
    if (ctx->precision == RT_FP64)
        launch_deposit64(g, ctx->bp64, view64(ctx, ctx->cur), ctx->perm, ctx->colstart, fdst, ctx->stream);
    else
        launch_deposit32(g, ctx->bp32, ctx->s32[ctx->cur], ctx->perm, ctx->colstart, fdst, ctx->car_ok, ctx->stream);
    prof_end(ctx);
    prof_begin(ctx, PC_DRAG);
    launch_drag(g, ctx->rho, ctx->coslat, fdst, ddst, ctx->stream);
    prof_end(ctx);
    HIP_OK(hipGetLastError());
    if (where == RT_HOST) {
        const size_t nf = (size_t)6 * (g.nz + 1) * g.ncol, nd = (size_t)2 * g.nz * g.ncol;
        if (flux) HIP_OK(hipMemcpyAsync(flux, fdst, sizeof(double) * nf, hipMemcpyDeviceToHost, ctx->stream));
        if (drag) HIP_OK(hipMemcpyAsync(drag, ddst, sizeof(double) * nd, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return RT_OK;
}

// a context scratch array allocated on first use
static rt_status ensure_scratch(rt_ctx ctx, double **p, size_t n)
{
    if (!*p) {
        *p = (double *)ctx_alloc(ctx, sizeof(double) * n);
        if (!*p) return rt_fail(ctx, RT_E_NOMEM, "no device memory for %zu doubles of scratch", n);
    }
    return RT_OK;
}

// copy a device result to the caller's pointer (host or device); no copy
// when the pointer is NULL
static rt_status hand_out(rt_ctx ctx, double *dst, const double *src, size_t n, int32_t where)
{
    if (!dst) return RT_OK;
    HIP_OK(hipMemcpyAsync(dst, src, sizeof(double) * n,
                          where == RT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, ctx->stream));
    return RT_OK;
}

extern "C" rt_status rt_full_fluxes(rt_ctx ctx, double *flux, double *tend, int32_t smooth, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    const size_t plane = (size_t)(g.nz + 1) * g.ncol, cells = (size_t)g.nz * g.ncol;
    rt_status st = ensure_scratch(ctx, &ctx->full, 8 * plane);
    if (!st) st = ensure_scratch(ctx, &ctx->fullt, 3 * cells);
    if (!st && smooth) st = ensure_scratch(ctx, &ctx->fulls, 8 * plane);
    if (st) return st;
    prof_begin(ctx, PC_DEPOSIT);
    if (ctx->precision == RT_FP64)
        launch_full_fluxes64(g, ctx->bp64, view64(ctx, ctx->cur), ctx->frow, ctx->perm, ctx->colstart, ctx->rho,
                             ctx->full, ctx->stream);
    else
        launch_full_fluxes32(g, ctx->bp32, ctx->s32[ctx->cur], ctx->frow32, ctx->perm, ctx->colstart, ctx->rho,
                             ctx->full, ctx->stream);
    const double *F = ctx->full;
    if (smooth) {
        launch_smooth(g, ctx->full, ctx->fulls, (int64_t)8 * (g.nz + 1), ctx->stream);
        F = ctx->fulls;
    }
    prof_end(ctx);
    prof_begin(ctx, PC_DRAG);
    launch_full_tend(g, ctx->coslat, ctx->rho, ctx->frow, F, ctx->fullt, ctx->stream);
    prof_end(ctx);
    HIP_OK(hipGetLastError());
    st = hand_out(ctx, flux, F, 8 * plane, where);
    if (!st) st = hand_out(ctx, tend, ctx->fullt, 3 * cells, where);
    if (st) return st;
    if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

extern "C" rt_status rt_budget(rt_ctx ctx, double *fields, double *terms, int32_t smooth, int32_t where)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const Grid &g = ctx->g;
    const size_t plane = (size_t)(g.nz + 1) * g.ncol, cells = (size_t)g.nz * g.ncol;
    rt_status st = ensure_scratch(ctx, &ctx->bud, 4 * plane);
    if (!st) st = ensure_scratch(ctx, &ctx->budt, 2 * cells);
    if (!st && smooth) st = ensure_scratch(ctx, &ctx->buds, 4 * plane);
    if (st) return st;
    prof_begin(ctx, PC_DEPOSIT);
    if (ctx->precision == RT_FP64)
        launch_budget64(g, ctx->bp64, view64(ctx, ctx->cur), ctx->perm, ctx->colstart, ctx->bud, ctx->stream);
    else
        launch_budget32(g, ctx->bp32, ctx->s32[ctx->cur], ctx->perm, ctx->colstart, ctx->bud, ctx->stream);
    const double *F = ctx->bud;
    if (smooth) {
        launch_smooth(g, ctx->bud, ctx->buds, (int64_t)4 * (g.nz + 1), ctx->stream);
        F = ctx->buds;
    }
    prof_end(ctx);
    prof_begin(ctx, PC_DRAG);
    launch_budget_terms(g, ctx->coslat, F, ctx->budt, ctx->stream);
    prof_end(ctx);
    HIP_OK(hipGetLastError());
    st = hand_out(ctx, fields, F, 4 * plane, where);
    if (!st) st = hand_out(ctx, terms, ctx->budt, 2 * cells, where);
    if (st) return st;
    if (where == RT_HOST) HIP_OK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

static rt_status read_counters(rt_ctx ctx, DevCounters *h)
{
    HIP_OK(hipMemcpyAsync(h, ctx->dc, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

extern "C" rt_status rt_get_rays(rt_ctx ctx, rt_rays *rays, int64_t *n_inout, int32_t where)
{
    if (!ctx || !n_inout) return rt_fail(ctx, RT_E_ARG, "n_inout is required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    if (!ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "no rays loaded");
    DevCounters h;
    rt_status st = read_counters(ctx, &h);
    if (st) return st;
    const int64_t n = h.n_active;
    if (*n_inout < n) {
        const long long have = (long long)*n_inout;
        *n_inout = n;
        return rt_fail(ctx, RT_E_ARG, "output arrays hold %lld, need %lld", have, (long long)n);
    }
    *n_inout = n;
    if (n == 0) return RT_OK;
    st = check_rays(ctx, rays);
    if (st) return st;
    rt_rays dst = *rays;
    void *staged = nullptr;
    if (where == RT_HOST) {
        st = stage_rays(ctx, &dst, n);
        if (st) return st;
        staged = dst.x;
    }
    if (ctx->precision == RT_FP64)
        launch_store64(ctx->g, view64(ctx, ctx->cur), ctx->perm, ctx->dc, dst, n, ctx->stream);
    else
        launch_store32(ctx->g, view32(ctx, ctx->cur), ctx->perm, ctx->dc, dst, n, ctx->stream);
    HIP_OK(hipGetLastError());
    if (where == RT_HOST) {
        double *hs[13] = {rays->x, rays->y, rays->z, rays->k, rays->l, rays->m, rays->dx,
                          rays->dy, rays->dz, rays->px, rays->py, rays->pz, rays->n};
        const double *ds[13] = {dst.x, dst.y, dst.z, dst.k, dst.l, dst.m, dst.dx, dst.dy, dst.dz, dst.px, dst.py, dst.pz, dst.n};
        for (int q = 0; q < 13; q++)
            HIP_OK(hipMemcpyAsync(hs[q], ds[q], sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipMemcpyAsync(rays->id, dst.id, sizeof(int64_t) * n, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (staged) unstage(ctx, staged);
    return RT_OK;
}

extern "C" rt_status rt_get_columns(rt_ctx ctx, uint32_t *cols, int64_t *n_inout, int32_t where)
{
    if (!ctx || !n_inout) return rt_fail(ctx, RT_E_ARG, "n_inout is required");
    if (where != RT_HOST && where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    if (!ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "no rays loaded");
    DevCounters h;
    rt_status st = read_counters(ctx, &h);
    if (st) return st;
    const int64_t n = h.n_active;
    if (*n_inout < n) {
        const long long have = (long long)*n_inout;
        *n_inout = n;
        return rt_fail(ctx, RT_E_ARG, "output array holds %lld, need %lld", have, (long long)n);
    }
    *n_inout = n;
    if (n == 0) return RT_OK;
    if (!cols) return rt_fail(ctx, RT_E_ARG, "cols is required");
    // the sorted keys of the active set are the columns in internal order
    HIP_OK(hipMemcpyAsync(cols, ctx->skeys, sizeof(uint32_t) * n,
                          where == RT_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

// the diagnostics without consuming the numeric-failure report
rt_status fill_stats(rt_ctx ctx, rt_stats *out)
{
    memset(out, 0, sizeof(*out));
    out->first_bad_id = -1;
    if (ctx->have_rays) {
        if (ctx->precision == RT_FP64)
            launch_stats64(view64(ctx, ctx->cur), ctx->perm, ctx->dc, ctx->red, ctx->n_bound, ctx->stream);
        else
            launch_stats32(ctx->s32[ctx->cur], ctx->perm, ctx->dc, ctx->red, ctx->n_bound, ctx->stream);
        HIP_OK(hipGetLastError());
        double sums[4];
        HIP_OK(hipMemcpyAsync(sums, ctx->red, sizeof(sums), hipMemcpyDeviceToHost, ctx->stream));
        DevCounters h;
        rt_status st = read_counters(ctx, &h);
        if (st) return st;
        out->n_active = h.n_active;
        out->n_top = h.removed[RK_TOP];
        out->n_bottom = h.removed[RK_BOTTOM];
        out->n_pole = h.removed[RK_POLE];
        out->n_invalid = h.removed[RK_INVALID];
        out->n_capped = h.removed[RK_CAPPED];
        out->n_merged = h.n_merged;
        out->n_split = h.n_split;
        out->sum_W = sums[0];
        out->sum_kW = sums[1];
        out->sum_lW = sums[2];
        out->sum_mW = sums[3];
        out->removed_W = h.removed_W;
        out->steps = h.steps;
        out->n_launched = h.n_launched;
        out->launched_W = h.launched_W;
        if (h.bad_key) out->first_bad_id = (int64_t)~h.bad_key;
    }
    return RT_OK;
}

extern "C" rt_status rt_get_stats(rt_ctx ctx, rt_stats *out)
{
    if (!ctx || !out) return rt_fail(ctx, RT_E_ARG, "out is required");
    rt_status st = fill_stats(ctx, out);
    if (st) return st;
    if (out->first_bad_id >= 0) {
        // reported once: the next report covers volumes deactivated after this call
        const uint64_t none = 0;
        HIP_OK(hipMemcpyAsync(&ctx->dc->bad_key, &none, sizeof(none), hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        return rt_fail(ctx, RT_E_NUMERIC, "ray volume id %lld (the smallest of those found) was non-finite or "
                       "degenerate and has been deactivated", (long long)out->first_bad_id);
    }
    return RT_OK;
}

extern "C" rt_status rt_split_merge(rt_ctx ctx, double alpha_split, int32_t n_max_per_cell, int32_t mode, rt_stats *out)
{
    if (!ctx) return RT_E_ARG;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (mode != RT_MERGE && mode != RT_CAP && mode != RT_SPLIT_ONLY) return rt_fail(ctx, RT_E_ARG, "bad mode");
    if (mode != RT_SPLIT_ONLY && n_max_per_cell < 1) return rt_fail(ctx, RT_E_ARG, "n_max_per_cell must be >= 1");
    ctx->car_ok = false;  // split pieces and merged volumes sit elsewhere
    return do_split_merge(ctx, alpha_split, n_max_per_cell, mode, out);
}

extern "C" rt_status rt_launch(rt_ctx ctx, const rt_launch_params *p, int64_t *n_launched)
{
    if (ctx) ctx->car_ok = false;  // launched volumes carry no carrier background
    if (!ctx) return RT_E_ARG;
    if (n_launched) *n_launched = 0;
    if (!ctx->have_bg || !ctx->have_rays) return rt_fail(ctx, RT_E_STATE, "background and rays are required");
    if (!p) return rt_fail(ctx, RT_E_ARG, "parameters are required");
    const Grid &g = ctx->g;
    if (!(p->dt > 0.0) || !std::isfinite(p->dt) || !(p->lambda_h > 0.0) || !std::isfinite(p->lambda_h) ||
        !(p->c_min >= 0.0) || !(p->c_max > p->c_min) || !std::isfinite(p->c_max) || !(p->c_width > 0.0) ||
        !std::isfinite(p->c_center) || !std::isfinite(p->t_solstice) || !(p->F_s >= 0.0) || !(p->F_w >= 0.0) ||
        !(p->z_launch > 0.0) || !(p->z_launch < g.Lz))
        return rt_fail(ctx, RT_E_ARG, "bad launch parameters");
    if (p->n_speeds < 1 || p->n_speeds > 64) return rt_fail(ctx, RT_E_ARG, "n_speeds must be 1 .. 64");
    if ((int64_t)g.ncol * 4 * p->n_speeds >= ((int64_t)1 << 31))
        return rt_fail(ctx, RT_E_UNSUPPORTED, "2^31 or more launch candidates (columns x 4 x n_speeds)");
    if (!p->flux_col && g.geometry != RT_SPHERICAL)
        return rt_fail(ctx, RT_E_ARG, "the box needs a launch flux per column");
    if (p->flux_col && p->where != RT_HOST && p->where != RT_DEVICE) return rt_fail(ctx, RT_E_ARG, "bad 'where'");
    const int64_t need = launch_scratch_len(g, p->n_speeds);
    if (need > ctx->lscr_len) {
        uint32_t *s = (uint32_t *)ctx_alloc(ctx, sizeof(uint32_t) * (size_t)need);
        if (!s) return rt_fail(ctx, RT_E_NOMEM, "no device memory for the launch scratch");
        ctx->lscr = s;
        ctx->lscr_len = need;
    }
    const double *flux_dev = nullptr;
    if (p->flux_col) {
        if (p->where == RT_DEVICE) {
            flux_dev = p->flux_col;
        } else {
            rt_status st = ensure_scratch(ctx, &ctx->lflux, (size_t)g.ncol);
            if (st) return st;
            HIP_OK(hipMemcpyAsync(ctx->lflux, p->flux_col, sizeof(double) * g.ncol, hipMemcpyHostToDevice,
                                  ctx->stream));
            flux_dev = ctx->lflux;
        }
    }
    int64_t cnt = 0;
    rt_status st = do_launch(ctx, p, flux_dev, ctx->lscr, &cnt);
    if (n_launched) *n_launched = st == RT_OK ? cnt : 0;
    return st;
}

// ---------------------------------------------------------------------------
// Allocation-free load from host memory (rt_set_rays_host_noalloc).  Where
// rt_set_rays(..., RT_HOST) allocates a device staging area for the host
// arrays on every call, this variant stages them through one fixed device
// array, `scratch`, one chunk of RT_NOALLOC_CHUNK volumes at a time (13
// doubles and an id per volume), and runs the same load kernels on each
// chunk.  Each GPU holds its own copy of the array until the process ends;
// its device address is looked up once per device and kept.  Calls that
// overlap on one GPU (two contexts on different streams) race on it.
// ---------------------------------------------------------------------------
#define NOALLOC_MAX_DEVICES 64
static_assert((size_t)RT_NOALLOC_CHUNK * 14 * sizeof(double) == RT_NOALLOC_SCRATCH_BYTES,
              "the staging chunk fills the scratch array");
static __device__ __align__(256) unsigned char scratch[RT_NOALLOC_SCRATCH_BYTES];
static std::mutex scratch_mu;
static void *scratch_ptr[NOALLOC_MAX_DEVICES];

// device address of `scratch` on the context's device (looked up with that
// device current, once per device)
static rt_status scratch_of(rt_ctx ctx, unsigned char **out)
{
    if (ctx->device < 0 || ctx->device >= NOALLOC_MAX_DEVICES)
        return rt_fail(ctx, RT_E_UNSUPPORTED, "device %d is beyond the %d this build tracks", ctx->device,
                       NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[ctx->device]) {
        int cur = -1;
        HIP_OK(hipGetDevice(&cur));
        if (cur != ctx->device) HIP_OK(hipSetDevice(ctx->device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != ctx->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return rt_fail(ctx, RT_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        scratch_ptr[ctx->device] = p;
    }
    *out = (unsigned char *)scratch_ptr[ctx->device];
    return RT_OK;
}

static S64 state_at(S64 s, int64_t off)
{
    double **f[13] = {&s.x, &s.y, &s.z, &s.k, &s.l, &s.m, &s.dx, &s.dy, &s.dz, &s.px, &s.py, &s.pz, &s.n};
    for (int q = 0; q < 13; q++) *f[q] += off;
    s.id += off;
    s.W += off;
    return s;
}

static S32 state_at(S32 s, int64_t off)
{
    float **f[11] = {&s.xi, &s.eta, &s.zeta, &s.k, &s.l, &s.dxi, &s.deta, &s.dz, &s.px, &s.py, &s.pz};
    for (int q = 0; q < 11; q++) *f[q] += off;
    s.col += off;
    s.lev += off;
    s.m += off;
    s.W += off;
    s.id += off;
    return s;
}

extern "C" rt_status rt_set_rays_host_noalloc(rt_ctx ctx, const rt_rays *rays, int64_t n)
{
    if (!ctx) return RT_E_ARG;
    if (n < 0) return rt_fail(ctx, RT_E_ARG, "negative ray count");
    if (n > ctx->cap) return rt_fail(ctx, RT_E_CAPACITY, "%lld ray volumes exceed capacity %lld", (long long)n,
                                     (long long)ctx->cap);
    if (n > 0) {
        rt_status st = check_rays(ctx, rays);
        if (st) return st;
    }
    unsigned char *stage = nullptr;
    rt_status st = scratch_of(ctx, &stage);
    if (st) return st;
    HIP_OK(hipMemsetAsync(ctx->dc, 0, sizeof(DevCounters), ctx->stream));
    ctx->cur = 0;
    ctx->hm_on = false;
    ctx->home = 0;
    for (int64_t off = 0; off < n; off += RT_NOALLOC_CHUNK) {
        const int64_t c = n - off < (int64_t)RT_NOALLOC_CHUNK ? n - off : (int64_t)RT_NOALLOC_CHUNK;
        // chunk layout in the scratch array: 13 fields of c doubles, then c ids
        // (a later chunk's copies are ordered after this chunk's kernels on
        // the stream)
        double *base = (double *)stage;
        rt_rays d;
        double **df[13] = {&d.x, &d.y, &d.z, &d.k, &d.l, &d.m, &d.dx, &d.dy, &d.dz, &d.px, &d.py, &d.pz, &d.n};
        const double *hs[13] = {rays->x, rays->y, rays->z, rays->k, rays->l, rays->m, rays->dx,
                                rays->dy, rays->dz, rays->px, rays->py, rays->pz, rays->n};
        for (int q = 0; q < 13; q++) {
            *df[q] = base + (int64_t)q * c;
            HIP_OK(hipMemcpyAsync(*df[q], hs[q] + off, sizeof(double) * (size_t)c, hipMemcpyHostToDevice, ctx->stream));
        }
        d.id = (int64_t *)(base + 13 * c);
        HIP_OK(hipMemcpyAsync(d.id, rays->id + off, sizeof(int64_t) * (size_t)c, hipMemcpyHostToDevice, ctx->stream));
        if (ctx->precision == RT_FP64)
            launch_load64(ctx->g, d, c, state_at(ctx->s64[0], off), ctx->key[0] + off, ctx->stream);
        else
            launch_load32(ctx->g, d, c, state_at(ctx->s32[0], off), ctx->key[0] + off, ctx->stream);
        launch_maxid(d.id, c, ctx->dc, ctx->stream);
        HIP_OK(hipGetLastError());
    }
    launch_set_sorted(ctx->dc, n, ctx->stream);
    ctx->n_bound = n;
    ctx->n_sorts = 0;
    st = sort_current(ctx);
    if (st) return st;
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->have_rays = true;
    ctx->car_ok = false;  // loaded volumes carry no carrier background
    return RT_OK;
}
