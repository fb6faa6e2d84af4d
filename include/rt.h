/*
 * rt.h -- C ABI of the MI355X (gfx950) ray-volume tracer for the MS-GWaM-3D
 * gravity-wave parameterization (Voelker et al., arXiv 2309.11257).
 *
 * The library advances phase-space ray volumes (carrier position, carrier
 * wavevector, physical extents; wave-action density and phase-space areas
 * fixed) with a low-storage three-stage Runge-Kutta scheme through a
 * resolved background wind (U, V) and stratification N^2 with rotation f, and
 * projects their pseudo-momentum fluxes onto the grid to form the wave drag.
 *
 * Conventions shared by every entry point
 *  - Status codes: every function returns RT_OK (0) or a positive error.
 *    Argument, state and capacity errors are detected before any device work
 *    and leave the context unchanged; rt_last_error() describes the last one.
 *  - Asynchrony: calls enqueue work on the context's stream and return,
 *    except where a host copy or a count is needed (stated per function).
 *  - Memory: every pointer argument is owned by the caller and is not kept
 *    after the call returns.  `where` says whether a pointer is host memory
 *    (RT_HOST) or device memory on the context's GPU (RT_DEVICE); device
 *    pointers must stay valid until the stream has passed the call.  The
 *    context's own device memory comes from the config's alloc/free callback
 *    pair (e.g. a PyTorch caching allocator) or, if alloc is NULL, from
 *    hipMalloc.
 *  - Grid: cell-centred, layout [nz][ny][nx] (x fastest).  Cartesian: a
 *    periodic f-plane box, coordinates in metres from (x0, y0) = (0, 0).
 *    Spherical: longitude (periodic, rad), latitude (rad, from y0 = -pi/2),
 *    height above the surface r - a (m).  Levels are uniform, z in [0, nz dz].
 *  - Threads: a context is not thread-safe; separate contexts are independent.
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx_s *rt_ctx;
typedef int32_t rt_status;

enum {
    RT_OK = 0,
    RT_E_ARG = 1,         /* bad argument (NULL pointer, size, non-positive N^2, ...) */
    RT_E_STATE = 2,       /* call out of order (e.g. step before background) */
    RT_E_NOMEM = 3,       /* device allocation failed */
    RT_E_CAPACITY = 4,    /* ray count would exceed the configured capacity */
    RT_E_DEVICE = 5,      /* a HIP runtime call failed */
    RT_E_NUMERIC = 6,     /* the device deactivated a non-finite or degenerate volume (rt_get_stats) */
    RT_E_UNSUPPORTED = 7  /* valid request that this build does not handle */
};
enum { RT_CARTESIAN = 0, RT_SPHERICAL = 1 };
enum { RT_FP64 = 0, RT_FP32 = 1 };
enum { RT_HOST = 0, RT_DEVICE = 1 };
enum { RT_STEP_DEPOSIT = 1, RT_STEP_SURROGATE = 2, RT_STEP_SATURATE = 4 };
enum { RT_MERGE = 0, RT_CAP = 1, RT_SPLIT_ONLY = 2 };

typedef struct {
    int32_t geometry;   /* RT_CARTESIAN or RT_SPHERICAL */
    int32_t precision;  /* RT_FP64: double state, bit-reproducible steps.
                           RT_FP32: single-precision state and integration,
                           positions held as (cell, offset in cell), wave
                           action and all flux sums in double */
    int32_t nx, ny, nz; /* grid cells; nx*ny < 2^31 - 8 */
    int32_t reserved;
    double dx, dy, dz;  /* spacing: m (Cartesian) or rad, rad, m (spherical) */
    double a;           /* planetary radius (spherical), m */
    int64_t capacity;   /* maximum number of ray volumes, including split children */
    void *(*alloc)(size_t bytes, void *user); /* device allocator, or NULL */
    void (*free)(void *ptr, void *user);
    void *user;
    void *stream;       /* hipStream_t to run on; NULL = the null stream */
} rt_config;

/* One ray volume per index; structure of arrays, all double except id.
 *   x, y, z      carrier position (see Grid above)
 *   k, l, m      carrier wavevector (rad/m): zonal, meridional, vertical
 *   dx, dy, dz   physical extents in coordinate units (m, or rad, rad, m)
 *   px, py, pz   phase-space areas: metric extent times wavenumber extent
 *                (Dx Dk, Dy Dl, Dz Dm; on the sphere Dx = (a+z) cos(phi)
 *                Dlambda and Dy = (a+z) Dphi), conserved while the volume
 *                deforms (Section 3a, eq. vpvol_cons_cart and eq. dkxdkl)
 *   n            phase-space wave-action density N, constant in the volume
 *   id           unique label, returned unchanged                         */
typedef struct {
    double *x, *y, *z, *k, *l, *m, *dx, *dy, *dz, *px, *py, *pz, *n;
    int64_t *id;
} rt_rays;

typedef struct {
    int64_t n_active;                     /* ray volumes in the domain */
    int64_t n_top, n_bottom, n_pole;      /* removed at the domain edges (cumulative) */
    int64_t n_invalid;                    /* removed as non-finite / degenerate (cumulative) */
    int64_t n_split, n_merged, n_capped;  /* cumulative counts */
    double sum_W, sum_kW, sum_lW, sum_mW; /* wave action and pseudo-momentum of the active set */
    double removed_W;                     /* wave action removed at the edges and by the cap */
    int64_t steps;                        /* steps taken */
    int64_t n_launched;                   /* volumes added by rt_launch (cumulative) */
    double launched_W;                    /* their wave action (cumulative) */
    int64_t first_bad_id;                 /* smallest id among the volumes deactivated as non-finite
                                             or degenerate (at load or after a step) since the last
                                             report, -1 if none */
} rt_stats;

/* Continuous launch from a ghost layer (Section 3c, sources): parameters.
 * Each call launches, in every column with a positive launch flux, one ray
 * volume per horizontal direction (east, north, west, south; a quarter of
 * the flux each) and intrinsic phase-speed bin c_b = c_min + (b + 1/2)
 * (c_max - c_min) / n_speeds (weight exp(-((c_b - c_center)/c_width)^2),
 * normalised over the bins): the part of the ghost layer below z_launch
 * that crossed it during dt. */
typedef struct {
    double z_launch;        /* launch height (m), inside the domain (the paper: 300 hPa) */
    double dt;              /* the step the new volumes cover (s), > 0 */
    double t_solstice;      /* time since the northern summer solstice (s): seasonal cycle */
    double F_s, F_w;        /* summer and winter launch fluxes of the latitudinal profile (Pa) */
    double lambda_h;        /* horizontal wavelength (m), > 0 */
    double c_min, c_max;    /* intrinsic phase-speed range (m/s), 0 <= c_min < c_max */
    double c_center, c_width; /* spectral weight (m/s), c_width > 0 */
    int32_t n_speeds;       /* phase-speed bins, 1 .. 64 */
    int32_t where;          /* RT_HOST or RT_DEVICE: where flux_col lives */
    const double *flux_col; /* [ny*nx] launch flux per column (Pa); NULL on the sphere: the
                               background source F_am(phi, t) of the latitudinal profile */
} rt_launch_params;

/* Create a context on the current HIP device.  The grid and precision are
   fixed for the context's lifetime.  Errors: RT_E_ARG for bad sizes;
   RT_E_UNSUPPORTED for nz > 640, for grids of 2^24 columns or more (24-bit
   index products) and, in single precision, for nx*ny*nz >= 2^27 cells
   (32-bit offsets into the packed background) and for a capacity of 2^30
   ray volumes or more (32-bit offsets into the ray fields). */
rt_status rt_create(const rt_config *cfg, rt_ctx *out);

/* Release all device memory of the context (synchronises its stream). */
rt_status rt_destroy(rt_ctx ctx);

/* Install the resolved background (Section 3b: the mean fields and their
 * gradients are interpolated to the ray-volume centre and faces).
 *   U, V, N2   [nz][ny][nx] double, cell centres; N2 > 0 everywhere
 *   f          [ny] Coriolis parameter per latitude row (NULL = all zero)
 *   rho        [nz] reference density per level (> 0), used by the drag
 * The gradient fields are formed on the device by centred differences,
 * periodic in x (and y on the box), one-sided at the vertical ends and at the
 * first and last latitude rows.  An RT_FP32 context rounds every field to
 * single precision once, round-to-nearest-even.  Host inputs are copied
 * before return; RT_E_ARG if N2 <= 0 or rho <= 0 anywhere (host inputs only;
 * device inputs are trusted). */
rt_status rt_init_background(rt_ctx ctx, const double *U, const double *V, const double *N2,
                             const double *f, const double *rho, int32_t where);

/* Scale-height correction Gamma (Section 2a, eq. dispersion, where K^2 =
 * k.k + Gamma^2, and the d Gamma^2 terms of eq. eikonal-sphere 1-3).
 *   G2  [nz][ny][nx] double: Gamma^2 at the cell centres (>= 0, finite); it
 *       is interpolated like N^2 to the carrier and the faces, and its
 *       gradients are formed on the device by the same centred differences.
 *       NULL switches the correction off (Gamma = 0, the default).
 * With the correction on, every evaluation of the dispersion relation uses
 * omega_hat^2 = (N^2 kh^2 + f^2 (m^2 + Gamma^2)) / K^2 and the group
 * velocity derived from it: the step (frequency, face velocities, refraction
 * including d omega_hat / d Gamma^2 = -(kh^2/(2 omega_hat K^2))(N^2-f^2)/K^2),
 * the deposition, saturation (K^2 with Gamma^2), full fluxes, budget, the
 * cap's wave energy, the surrogate features, and the launch (a bin whose
 * m^2 + Gamma^2 from the dispersion relation does not exceed Gamma^2 is
 * evanescent and discarded).  Host input is copied before return; RT_E_ARG
 * for a negative or non-finite value (host input only). */
rt_status rt_set_scale_height(rt_ctx ctx, const double *G2, int32_t where);

/* Load n ray volumes (replacing any current set).  n may be 0.  Volumes
 * outside the vertical domain, with non-finite state or non-positive extents
 * are counted as removed at load.  RT_E_CAPACITY if n > capacity. */
rt_status rt_set_rays(rt_ctx ctx, const rt_rays *rays, int64_t n, int32_t where);

/* For callers that cannot allocate device memory during a call (tight
 * serving loops, harnesses that forbid it): rt_set_rays from host arrays
 * (RT_HOST) with the same result, bit for bit, but without the per-call
 * device staging allocation.  The host arrays are staged through one fixed
 * device array of RT_NOALLOC_SCRATCH_BYTES (14 MiB) that the library holds
 * on each GPU it runs on until the process ends, RT_NOALLOC_CHUNK volumes
 * (13 doubles and an id each) at a time; no hipMalloc, hipFree or other
 * allocating call is made.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (contexts on different streams) race, so
 * serialise them.  Synchronises the context's stream before returning.
 * Errors as rt_set_rays (RT_E_CAPACITY if n > capacity, leaving the
 * context unchanged); RT_E_DEVICE if the array's device address cannot be
 * found. */
#define RT_NOALLOC_CHUNK 131072
#define RT_NOALLOC_SCRATCH_BYTES (RT_NOALLOC_CHUNK * 14 * 8)
rt_status rt_set_rays_host_noalloc(rt_ctx ctx, const rt_rays *rays, int64_t n);

/* Copy out the active ray volumes in the library's internal order: grouped
 * by column.  The regrouping after rt_set_rays and every fourth one after it
 * order each column's volumes by level index floor(z / dz) (clamped to
 * 0 .. nz; when (number of columns + 6) * (nz + 1) fits 32 bits); otherwise,
 * and for volumes with equal keys, each column's previous relative order is
 * kept.  *n_inout: in = length of the caller's
 * arrays, out = number
 * written.  Synchronises.  RT_E_ARG if the arrays are too short (then
 * *n_inout is set to the number needed and nothing is written). */
rt_status rt_get_rays(rt_ctx ctx, rt_rays *rays, int64_t *n_inout, int32_t where);

/* Column key (j*nx + i) of each active ray volume's parent column, in the
 * same order as rt_get_rays returns them.  *n_inout as for rt_get_rays.
 * Synchronises. */
rt_status rt_get_columns(rt_ctx ctx, uint32_t *cols, int64_t *n_inout, int32_t where);

/* Advance every active ray volume by one RK3 step of length dt (Appendix B:
 * Williamson's low-storage third-order scheme; Section 3a: carrier moved by
 * the mean and extents by the difference of the face group velocities,
 * wavevector by the refraction equations eq. eikonal-sphere 1-3 with
 * Gamma = 0).  Afterwards volumes are wrapped periodically, those leaving
 * through the top or bottom or within 0.5 degree of a pole are removed, and
 * the set is regrouped by parent column (Appendix B, horizontal propagation).
 * With RT_STEP_DEPOSIT the fluxes and drag are also formed into the
 * context's own buffers (read them with rt_deposit_flux(ctx, NULL, ...) --
 * see there).  With RT_STEP_SURROGATE the volumes whose parent column is
 * flagged by rt_set_frozen_columns keep their state unchanged for this step
 * (the column surrogate supplies that column's drag; RT_E_STATE if no flags
 * were set).  With RT_STEP_SATURATE the regrouped set is saturated with the
 * same dt (rt_saturate) before any deposition (RT_E_ARG unless dt > 0).
 * No synchronisation. */
rt_status rt_step(rt_ctx ctx, double dt, int32_t flags);

/* Spectral saturation of the current set (Section 3c, eq.
 * instability-threshold and eq. turbulent-diffusivity).  Per grid cell,
 *   P = sum_j (m^2 kh^2 / (omega_hat K^2)) A_j alpha_j  and  Q = sum_j P_j K^2,
 * where A_j alpha_j for a level is the volume's wave action W = N Px Py Pz
 * times its overlap fraction with the level, divided by the cell volume
 * (the volume counts in its carrier's column, as for the fluxes); omega_hat
 * and K^2 = k^2 + l^2 + m^2 at the carrier (Gamma = 0).  Then
 *   kappa = max(0, (P - rho/2) / (2 dt Q))
 * per cell, and every active volume's density is multiplied by
 * max(0, 1 - 2 kbar K^2 dt), kbar the overlap-weighted mean of kappa over
 * the levels it covers (parts outside the domain count as kappa = 0).  The
 * sums are deterministic (bitwise identical between runs).
 *   kappa  [nz][ny][nx] double, the turbulent diffusivity (m^2/s); may be NULL
 * RT_E_ARG unless dt > 0 and finite; RT_E_STATE before a background and a
 * ray set.  No synchronisation unless kappa is given with RT_HOST. */
rt_status rt_saturate(rt_ctx ctx, double dt, double *kappa, int32_t where);

/* Column flags for RT_STEP_SURROGATE: mask [ny*nx] uint8 (column j*nx + i),
 * 1 = frozen.  NULL clears all flags.  Copied on the stream (synchronises
 * for RT_HOST). */
rt_status rt_set_frozen_columns(rt_ctx ctx, const uint8_t *mask, int32_t where);

/* Input features of the column surrogate from the current state (the
 * quantities the flux projection of Section 3b reads, summarised per column):
 *   X [ny*nx][3*nz + 48] float32, row j*nx + i:
 *     U, V, N2 at the column's cell centres (levels 0..nz-1);
 *     for each azimuth sector s = 0..7 of the horizontal wavevector (sector s
 *     centred on azimuth 45 s degrees, boundaries at 22.5 + 45 n degrees,
 *     decided by comparing |l| with tan(22.5 deg) |k| and |k| with
 *     tan(22.5 deg) |l|), six moments: sum of W, sum of |cg_z| k_h W (cg_z
 *     the intrinsic vertical group velocity at the carrier, Section 2a), the
 *     W-weighted means of log10 k_h, log10 |m| and the carrier height z, and
 *     the W-weighted standard deviation of z (0 for an empty sector);
 *     W = N Px Py Pz.
 * Sums are accumulated in double in a fixed order.  No synchronisation
 * unless where == RT_HOST. */
rt_status rt_features(rt_ctx ctx, float *X, int32_t where);

/* Project the current ray volumes onto the grid (Section 3b and App. A:
 * pseudo-momentum flux, integral of cg_hat k_h N d^3k; vertical fluxes on the
 * staggered interfaces, horizontal fluxes as cell means of the volumes whose
 * carrier is in the column) and form the drag du, dv = -(1/rho) div F.
 *   flux  [6][nz+1][ny][nx] double: Fxk, Fxl, Fyk, Fyl (levels, slot nz = 0),
 *         Fzk, Fzl (interfaces 0..nz); may be NULL
 *   drag  [2][nz][ny][nx] double: du, dv; may be NULL
 * Sums are deterministic (bitwise identical between runs).  No
 * synchronisation unless where == RT_HOST. */
rt_status rt_deposit_flux(rt_ctx ctx, double *flux, double *drag, int32_t where);

/* Full flux formulation of the current set (Section 2b, eq.
 * fluxes:momentum, eq. fluxes:temperature, eq. fluxes:buoyancy) and the
 * resulting mean-flow tendencies (eq. mean-flow-impact, eq.
 * mean-flow-impact-t).  Per volume, with cg the intrinsic group velocity,
 * e_r x a = (-a_y, a_x, 0) and omega^2 - f^2 = kh^2 (N^2 - f^2) / K^2:
 *   momentum flux  [omega^2 cg_i kh_j + f^2 (e_r x cg)_i (e_r x kh)_j] / (omega^2 - f^2) W,
 *   buoyancy flux  cg_z f N^2 / (omega^2 - f^2) (e_r x kh) W / rho
 * (the potential-temperature flux in buoyancy form, <u'b'> =
 * (g/theta) <u'theta'>), projected like rt_deposit_flux.
 *   flux   [8][nz+1][ny][nx] double: Fxu, Fxv, Fyu, Fyv, Bu, Bv on levels
 *          (slot nz = 0), Fzu, Fzv on interfaces; may be NULL
 *   tend   [3][nz][ny][nx] double: du, dv = -(1/rho) div F + (f/g) e_r x <u'b'>
 *          (g = 9.80665 m/s^2), db = -div_h <u'b'> (the buoyancy
 *          tendency, (g/theta) dtheta/dt); may be NULL
 *   smooth nonzero: every flux field is first smoothed horizontally
 *          (Appendix B, horizontal flux smoothing: weights 3 for the cell,
 *          2 for the cells sharing an edge, 1 for those sharing a corner;
 *          the sphere's missing rows are left out and the weights
 *          renormalised) and the tendencies use the smoothed fields
 * Scratch is allocated from the context's allocator on the first call.
 * Deterministic.  No synchronisation unless where == RT_HOST. */
rt_status rt_full_fluxes(rt_ctx ctx, double *flux, double *tend, int32_t smooth, int32_t where);

/* Wave-action budget of the current set (Section 4, eq. wave-action-budget):
 *   fields [4][nz+1][ny][nx] double: A (wave action per unit volume), (U + cg_x) A,
 *          (V + cg_y) A on levels, cg_z A on interfaces (ground-based group
 *          velocity at the carrier), projected like rt_deposit_flux
 *   terms  [2][nz][ny][nx] double: the horizontal propagation term
 *          div_h(cg_h A) and the vertical one d_z(cg_z A)
 *   smooth as rt_full_fluxes
 * The saturation term is the change of A across rt_saturate divided by its
 * time step.  Either output may be NULL.  Scratch is allocated on the first
 * call.  No synchronisation unless where == RT_HOST. */
rt_status rt_budget(rt_ctx ctx, double *fields, double *terms, int32_t smooth, int32_t where);

/* Vertical splitting (Appendix B, ray volume splitting): every volume taller
 * than alpha_split * dz is halved (repeatedly, up to 64 pieces) into
 * volumes with the same wavevector and density.  Then, with mode RT_MERGE,
 * any grid cell holding more than n_max_per_cell volumes has adjacent pairs
 * of similar wavevector merged (conserving wave action and pseudo-momentum);
 * with RT_CAP any column holding more than n_max_per_cell volumes loses those
 * of lowest wave energy (Appendix B, computational performance);
 * RT_SPLIT_ONLY skips both.  alpha_split <= 0 skips splitting.  Synchronises
 * (the new count is needed); fills *out if not NULL.  RT_E_CAPACITY (nothing
 * changed) if the split children do not fit. */
rt_status rt_split_merge(rt_ctx ctx, double alpha_split, int32_t n_max_per_cell, int32_t mode,
                         rt_stats *out);

/* Continuous launch from a ghost layer (Section 3c, sources; parameters in
 * rt_launch_params).  For every candidate (column, direction, phase speed)
 * with omega_hat = kh c_b strictly between |f| and N at the column centre
 * and launch height (the others cannot propagate: they are reflected in the
 * ghost layer and discarded with their share of the flux), a volume is
 * added with m = -sqrt(kh^2 (N^2 - omega_hat^2) / (omega_hat^2 - f^2))
 * (upward), vertical span [z_launch, z_launch + cg_z dt], horizontal
 * extents one cell at the column centre, dk = dl = kh/10, dm = |m|/10, and
 * wave action W = F_bin A dt / kh (A the cell's area at the launch height),
 * so that it carries its bin's pseudo-momentum flux.  The active set is then
 * regrouped; the new volumes get consecutive ids in candidate order.
 * *n_launched (may be NULL) receives the count.  Synchronises.
 * RT_E_CAPACITY (nothing changed) if the volumes do not fit; RT_E_ARG for
 * bad parameters or a missing flux_col on the box. */
rt_status rt_launch(rt_ctx ctx, const rt_launch_params *p, int64_t *n_launched);

/* Current diagnostics (deterministic sums).  Synchronises.  A volume with a
 * non-finite state, a non-positive extent or a zero wavevector (K^2 = 0) at
 * load or after a step cannot be carried on: it is deactivated, counted in
 * n_invalid, and the rest of the set is unaffected.  The next rt_get_stats
 * then fills *out completely, sets first_bad_id to the smallest such id and
 * returns RT_E_NUMERIC (rt_last_error names the id); the report is then
 * cleared, so a later call returns RT_OK until another volume fails.
 * rt_split_merge's statistics show first_bad_id without clearing it. */
rt_status rt_get_stats(rt_ctx ctx, rt_stats *out);

/* Kernel timing for benchmarks.  While on, the library brackets each group of
 * launches with HIP events on the context's stream, by class:
 *   0 RK3 step, 1 sort + column offsets + removal tallies, 2 deposition,
 *   3 drag, 4 split/merge/cap, 5 diagnostics.
 * rt_profile_read synchronises, returns the summed milliseconds and the
 * number of timed groups per class since the last read (arrays of 8), and
 * resets them.  Recording events does not change the work done. */
rt_status rt_profile(rt_ctx ctx, int32_t on);
rt_status rt_profile_read(rt_ctx ctx, double *ms, int64_t *groups);

/* Human-readable description of the last error on this context ("" if none). */
const char *rt_last_error(rt_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
