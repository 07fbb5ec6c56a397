/* surrogate.h -- C ABI of the learned warm start (libpic.so).
 *
 * A surrogate maps the four quantities the paper varies or fixes per run --
 * emission flux Gamma ("Benchmark cases", Table 2), cathode temperature T_c,
 * bias V and neutral density n_g ("Model", "Emission and collisions") -- to
 * the late-time state on X cell centres: the profiles the paper reports
 * ("Results": time-averaged potential and densities) and, per species, the
 * shape of the late-time velocity distribution:
 *     out[b][0][x] = phi / V,  out[b][1][x] = ln(n_e / n0),  out[b][2][x] = ln(n_i / n0),
 *     out[b][3..11][x], out[b][12..20][x]: electron v_z and |v_perp| quantiles / sqrt(e / m_e),
 *     out[b][21..29][x], out[b][30..38][x]: ion v_z and |v_perp| quantiles / sqrt(e / m_i),
 * quantiles at the levels of pic_init_from_state (speeds in units of the
 * 1 eV thermal speed).  sur_state turns them into the state that
 * pic_init_from_state loads, so that a run starts near its late state.  The
 * paper has no surrogate; the network is a reading: six 1D convolutions
 * (kernel 5, zero padding 2) with channels 16 -> 64 (x5) -> 39 (padded to 48
 * on the matrix cores) and tanh between layers, on bfloat16 weights and activations with FP32
 * accumulation (gfx950 matrix cores), trained by mean squared error with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
 *
 * Input channels: the parameters mapped to [-1, 1] over Gamma in
 * [1e19, 1.2e20] m^-2 s^-1 (log), T_c in [1800, 2200] K, V in [5, 20] V,
 * n_g in [1e21, 1e22] m^-3 (log), and 12 functions of the position
 * u = (x + 1/2) / X: 2u - 1, 1 - 2u, sin / cos of (pi, 2 pi, 4 pi) u,
 * exp(-64 u), exp(-64 (1 - u)), exp(-16 u), exp(-16 (1 - u)).
 *
 * Packed weights (host arrays, FP32): layer by layer, W_l[co][ci][t] (t the
 * kernel tap, y[x] += W[co][ci][t] a[ci][x + t - 2]) -- SUR_WEIGHTS values --
 * and the biases b_l[co] -- SUR_BIASES values.
 *
 * Ownership: the caller owns the device workspace and the stream; the
 * library owns the host-side handle.  Errors: every call returns 0 or a
 * negative PIC_* code (pic.h); sur_last_error() has the message.  Calls on a
 * handle are asynchronous on its stream unless they say otherwise.
 */
#ifndef PAPER_2605_07083_SURROGATE_H
#define PAPER_2605_07083_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SUR_LAYERS 6
#define SUR_IN 16
#define SUR_HIDDEN 64
#define SUR_OUT 39
#define SUR_KS 5
#define SUR_WEIGHTS 99520   /* 64*16*5 + 4*64*64*5 + 39*64*5 */
#define SUR_BIASES 359      /* 5*64 + 39 */

typedef struct sur_net sur_net;

/* Device workspace for batches of up to max_batch samples of `cells`
 * positions (cells a positive multiple of 64). */
int sur_workspace_size(int max_batch, int cells, size_t *bytes);

/* Create a network over a caller-owned workspace (256-byte aligned) bound to
 * hip_stream.  Weights start N(0, 1/(5 C_in)) from Philox keyed by seed,
 * biases 0, Adam moments 0. */
int sur_create(int max_batch, int cells, void *dev_workspace, size_t bytes, void *hip_stream, uint32_t seed,
               sur_net **out);

/* Replace the master weights (host arrays, packed as above) and reset the Adam
 * moments and step count.  Synchronises. */
int sur_set_weights(sur_net *n, const float *w, const float *b);

/* Copy the master weights out (packed).  Synchronises. */
int sur_get_weights(sur_net *n, float *w, float *b);

/* Gradients of the mean squared error from the last sur_train_step (packed).
 * Synchronises. */
int sur_get_grads(sur_net *n, float *w, float *b);

/* Forward pass.  dev_params [batch][4] = (Gamma, T_c K, V, n_g) FP32 on the
 * device; dev_out [batch][SUR_OUT][cells] FP32 on the device. */
int sur_forward(sur_net *n, const float *dev_params, int batch, float *dev_out);

/* sur_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same output bit for bit, with the activations in a
 * library-held static device array of 12 MiB per GPU instead of the handle's
 * workspace, so any batch size runs (in chunks of samples that fit it: 8
 * samples of 2048 cells).  Allocates nothing: no hipMalloc, hipFree or
 * allocating library call.  The handle's GPU must be current (PIC_EINVAL
 * otherwise); cells beyond 17096 per sample do not fit the array and are
 * refused (PIC_EINVAL).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (on different streams, or from several threads)
 * race and must be ordered by the caller.  Asynchronous on the handle's
 * stream. */
int sur_forward_noalloc(sur_net *n, const float *dev_params, int batch, float *dev_out);

/* One training step on a batch: forward, loss = mean over (b, c, x) of
 * (out - target)^2, backward (input and weight gradients on the matrix
 * cores; the gradient entering each layer rounded to bfloat16), one Adam
 * update of every master weight and bias, re-quantisation to bfloat16.
 * dev_target [batch][SUR_OUT][cells] FP32.  If loss != NULL the call synchronises
 * and stores the loss of this batch before the update. */
int sur_train_step(sur_net *n, const float *dev_params, const float *dev_target, int batch, float lr,
                   double *loss);

/* Forward pass converted to the warm-start loader's input: dev_dens
 * [batch][2][cells] doubles, n0[b] exp(out[b][1]) and n0[b] exp(out[b][2]);
 * dev_n0 [batch] doubles on the device. */
int sur_densities(sur_net *n, const float *dev_params, const double *dev_n0, int batch, double *dev_dens);

/* Message of the last failing surrogate call on this thread. */
/* The loader's state for a batch: dev_state [batch][39][cells] doubles with
 * row 0 n0 exp(out[1]), row 1 n0 exp(out[2]) (m^-3), row 2 V out[0] (V, with
 * V = params[b][2]) and rows 3..38 the quantile channels times their 1 eV
 * speeds (m/s): the layout pic_init_from_state reads (PIC_STATE_ROWS rows,
 * cells = N).  dev_n0: [batch] doubles.  Asynchronous. */
int sur_state(sur_net *n, const float *dev_params, const double *dev_n0, int batch, double *dev_state);

const char *sur_last_error(void);

/* Release the handle (not the caller's workspace or stream). */
void sur_destroy(sur_net *n);

#ifdef __cplusplus
}
#endif

#endif
