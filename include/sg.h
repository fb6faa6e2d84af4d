/*
 * sg.h -- C ABI of the column surrogate that accompanies the MI355X ray-volume
 * tracer (include/rt.h): a multilayer perceptron mapping a column's resolved
 * background profiles and coarse ray-spectrum moments to the column's wave-drag
 * profile, trained on data the tracer itself produces.  The paper has no
 * learned component; the tracer (Sections 2-3, Appendix B) is the reference
 * and the fallback wherever the surrogate is not trusted.
 *
 * Network: n_in -> n_hidden (x n_layers, GELU with the tanh form of
 * Hendrycks & Gimpel 2016) -> n_out, weights and activations in bfloat16,
 * products accumulated in float32 on the MFMA units (hand-written kernels,
 * v_mfma_f32_32x32x16_bf16), float32 master weights, Adam (Kingma & Ba 2015).
 * An ensemble of n_members independently initialised networks share the
 * shapes; their spread drives the trust gate.
 *
 * Conventions as in rt.h: status codes, caller-owned pointers, device
 * pointers on the net's GPU unless a `where` argument says RT_HOST, work
 * enqueued on the net's stream.  bfloat16 values are passed as uint16_t
 * (the upper half of the float32 bit pattern, round-to-nearest-even).
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#include "rt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_net_s *sg_net;

typedef struct {
    int32_t n_members;  /* ensemble size (>= 1) */
    int32_t n_in;       /* features per column (e.g. 3*nz + 32) */
    int32_t n_hidden;   /* width of the hidden layers */
    int32_t n_layers;   /* number of hidden layers (>= 1) */
    int32_t n_out;      /* outputs per column (e.g. 2*nz) */
    int32_t max_batch;  /* largest batch a call may pass */
    uint64_t seed;      /* weight initialisation (He-uniform, counter-based) */
    void *(*alloc)(size_t bytes, void *user); /* device allocator, or NULL for hipMalloc */
    void (*free)(void *ptr, void *user);
    void *user;
    void *stream;       /* hipStream_t */
} sg_config;

/* Create the ensemble with freshly initialised weights.  RT_E_ARG for bad
   shapes. */
rt_status sg_create(const sg_config *cfg, sg_net *out);
rt_status sg_destroy(sg_net net);

/* Number of float32 parameters of one member (all weights then biases, layer
 * by layer: W1[n_hidden][n_in], b1, W2, b2, ..., Wout[n_out][n_hidden], bout). */
int64_t sg_param_count(sg_net net);

/* Copy one member's float32 master parameters out / in (host or device).  Setting
 * parameters resets that member's Adam moments and step count. */
rt_status sg_get_params(sg_net net, int32_t member, float *params, int32_t where);
rt_status sg_set_params(sg_net net, int32_t member, const float *params, int32_t where);

/* Forward pass of one member (member >= 0) or of all members (member = -1).
 *   X  [B][n_in] bfloat16, device, standardised features
 *   Y  [B][n_out] float32 (one member) or [n_members][B][n_out] (all), device
 * No synchronisation. */
rt_status sg_forward(sg_net net, int32_t member, const uint16_t *X, float *Y, int32_t B);

/* One Adam step of one member on the mean-squared error
 * L = mean over the batch and outputs of (Y - T)^2.
 *   T     [B][n_out] float32 targets, device
 *   loss  float32 on the device receiving L (may be NULL)
 * lr is the Adam step size; beta1 = 0.9, beta2 = 0.999, eps = 1e-8. */
rt_status sg_train_step(sg_net net, int32_t member, const uint16_t *X, const float *T, int32_t B, float lr,
                        float *loss);

/* Gradient of L with respect to one member's parameters, without updating
 * anything (checking aid): grads has sg_param_count entries (host or device). */
rt_status sg_gradient(sg_net net, int32_t member, const uint16_t *X, const float *T, int32_t B, float *grads,
                      int32_t where);

/* Trust gate over columns.  A column is trusted (mask 1) when the ensemble's
 * spread -- the root-mean-square over outputs of the members' sample standard
 * deviation (n - 1 normalisation; 0 for one member) -- is at most tau and every feature lies within [fmin, fmax] of
 * the training data; otherwise it goes back to the ray tracer (mask 0).
 *   Yens  [n_members][n_cols][n_out] float32 (from sg_forward, member = -1)
 *   Xraw  [n_cols][n_in] float32 unstandardised features
 *   fmin, fmax  [n_in] float32; spread [n_cols] float32 output (may be NULL)
 *   mask  [n_cols] uint8 output
 * All device pointers. */
rt_status sg_gate(sg_net net, const float *Yens, const float *Xraw, const float *fmin, const float *fmax,
                  int32_t n_cols, float tau, float *spread, uint8_t *mask);

/* Network input from raw features: X[c][f] = bf16((T(x) - mean[f]) / std[f])
 * with T(x) = log10(max(x + logfloor[f], 1e-30)) where logfloor[f] > 0 and
 * T(x) = x where logfloor[f] == 0.
 *   Xraw [n_cols][n_in] float32; mean, std, logfloor [n_in] float32;
 *   X [n_cols][n_in] bfloat16 output.  All device pointers. */
rt_status sg_standardize(sg_net net, const float *Xraw, const float *mean, const float *std, const float *logfloor,
                         int32_t n_cols, uint16_t *X);

/* Training targets from the tracer's drag: T[c][o] = (drag[o][c] - mean[o]) /
 * std[o] for outputs o = comp*nz + k (n_out must equal 2*nz).
 *   drag [2][nz][n_cols] float64 (rt_deposit_flux layout); mean, std [n_out]
 *   float32; T [n_cols][n_out] float32 output.  All device pointers. */
rt_status sg_targets(sg_net net, const double *drag, const float *mean, const float *std, int32_t n_cols, int32_t nz,
                     float *T);

/* Replace the tracer's drag in trusted columns by the surrogate's: for every
 * column c with mask[c] = 1 and output o = comp*nz + k (n_out must equal
 * 2*nz), drag[o][c] = mean over members of (Yens[m][c][o] * std[o] + mean[o]).
 * Untrusted columns are left as they are.
 *   Yens [n_members][n_cols][n_out] float32; mean, std [n_out] float32;
 *   mask [n_cols] uint8; drag [2][nz][n_cols] float64 (the layout of
 *   rt_deposit_flux's drag, columns j*nx + i).  All device pointers.
 * RT_E_UNSUPPORTED for n_out > 256. */
rt_status sg_apply_drag(sg_net net, const float *Yens, const float *mean, const float *std, const uint8_t *mask,
                        int32_t n_cols, int32_t nz, double *drag);

/* Message of the last failed call on this net (static storage of the net). */
const char *sg_last_error(sg_net net);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */
