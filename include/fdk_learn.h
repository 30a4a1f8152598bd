/*
 * fdk_learn.h -- C ABI of the learned row filter: a data-driven replacement
 * for (or correction to) the ramp filter of the FDK pre-processing step, which
 * the paper takes as given (its input is filtered projections, Sections 2.1.2
 * and 3.1.1), trained through the back-projector of fdk.h.
 *
 * The filter network maps one cosine-weighted detector row (1 channel) to a
 * filtered row through 1-D convolutions along the row (u, the fastest axis of
 * a projection); the building blocks here are the layer operations, their
 * gradients, the squared-error loss of a reconstruction and an Adam update.
 *
 * Conventions (in addition to those of fdk.h)
 *   - activations   float32 [rows][channels][len], row-major: the `len`
 *                   samples of one channel of one row are contiguous.
 *   - weights       float32 [cout][cin][9], bias float32 [cout].
 *   - convolution   cross-correlation with 9 taps and 4 zeros of padding on
 *                   each side, so the output has the input's length:
 *                   out[r][o][x] = bias[o] + sum_i sum_t w[o][i][t] in[r][i][x+t-4]
 *   - channels      cin and cout each 1 or 32; anything else is
 *                   FDK_E_UNSUPPORTED.
 *   - all pointers are device memory on the current device, owned by the
 *     caller; distinct arguments must not overlap unless stated.  Work is
 *     enqueued on `stream` and is asynchronous.  Host-detectable errors are
 *     returned before any HIP call.
 */
#ifndef FDK_LEARN_H
#define FDK_LEARN_H

#include <stdint.h>

#include "fdk.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * fdk_cosine_weight -- step 1 of the FDK filter alone (the learned filter's
 * input):  out = raw * sdd / sqrt(sdd^2 + u_mm^2 + v_mm^2), with u_mm, v_mm as
 * in fdk_filter.  raw, out: device float32 [np][nh][nw] (sg->dtype FDK_F32);
 * out may equal raw (in place).
 */
fdk_status fdk_cosine_weight(const fdk_stack* sg, const float* raw, float* out, double du,
                             double dv, double sdd, double u_off, double v_off, void* stream);

/*
 * fdk_conv1d_forward -- one layer:
 *   y = bias + conv(in, w);  y = max(y, 0) if relu;  y = 0 where mask <= 0;
 *   out = alpha y + add.
 * in [rows][cin][len]; out, mask, add [rows][cout][len]; bias [cout].
 * bias, mask and add may be NULL (no bias / no mask / no addend).  `add` may
 * equal `out` (accumulate into out); `in` must not overlap `out`.
 */
fdk_status fdk_conv1d_forward(int32_t cin, int32_t cout, int32_t rows, int32_t len,
                              const float* in, const float* w, const float* bias,
                              const float* mask, const float* add, float alpha, int32_t relu,
                              float* out, void* stream);

/*
 * fdk_conv1d_backward_data -- gradient of a layer's loss with respect to its
 * input (transposed convolution), times an optional mask:
 *   gin[r][i][x] = [mask > 0] * sum_o sum_t w[o][i][t] gout[r][o][x-t+4]
 * gout [rows][cout][len]; gin, mask [rows][cin][len] (mask may be NULL;
 * passing the previous layer's ReLU output applies the ReLU derivative).
 * gin is overwritten.
 */
fdk_status fdk_conv1d_backward_data(int32_t cin, int32_t cout, int32_t rows, int32_t len,
                                    const float* gout, const float* w, const float* mask,
                                    float* gin, void* stream);

/*
 * fdk_conv1d_backward_weight -- gradients of a layer's weights and bias,
 * ACCUMULATED into gw [cout][cin][9] and gb [cout] (gb may be NULL):
 *   gw[o][i][t] += sum_r sum_x gout[r][o][x] in[r][i][x+t-4]
 *   gb[o]       += sum_r sum_x gout[r][o][x]
 * Uses float atomics: the last bits depend on the summation order.
 */
fdk_status fdk_conv1d_backward_weight(int32_t cin, int32_t cout, int32_t rows, int32_t len,
                                      const float* in, const float* gout, float* gw, float* gb,
                                      void* stream);

/*
 * fdk_sqerr -- squared-error loss of a reconstruction and its gradient:
 *   loss[0] += sum_q (a[q] - b[q])^2   (device float32 scalar, accumulated)
 *   grad[q]  = grad_scale * (a[q] - b[q])    (if grad is not NULL)
 * grad_scale = 2/n gives the gradient of the mean.  a, b, grad: n floats.
 */
fdk_status fdk_sqerr(int64_t n, const float* a, const float* b, float* grad, float grad_scale,
                     float* loss, void* stream);

/*
 * fdk_adam -- one Adam update (Kingma and Ba, ICLR 2015, Algorithm 1) of n
 * parameters p with gradient g and moments m, v (all device float32 [n], m
 * and v start at zero), at step t >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 */
fdk_status fdk_adam(int32_t n, float* p, const float* g, float* m, float* v, float lr,
                    float beta1, float beta2, float eps, int32_t t, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FDK_LEARN_H */
