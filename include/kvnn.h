/*
 * kvnn: a small 3-D convolutional network that predicts the steady state of
 * the laterally heated cube at a given Grashof number, to be used as the
 * initial guess of Newton's method.  The paper (Sec. 1) reaches steady states
 * at large Gr by Newton continuation, starting each solve from the state at a
 * nearby smaller Gr; the network is trained on such states and offers a
 * guess at Gr values it has not seen.  It is an addition to the paper's
 * method: the Newton residual of kv.h judges every guess it produces.
 *
 * Network (U-Net, three levels):
 *   inputs  4 channels on an r^3 grid of cell centres:
 *           2 xc - 1, 2 yc - 1, 2 zc - 1, (log10 Gr - m) / s
 *           with m = (lgr_lo + lgr_hi) / 2, s = (lgr_hi - lgr_lo) / 2;
 *   encoder conv3(4->16) conv3(16->16) | pool | conv3(16->32) conv3(32->32)
 *           | pool | conv3(32->64) conv3(64->64);
 *   decoder up, concat with level 2: conv3(96->32) conv3(32->32);
 *           up, concat with level 1: conv3(48->16) conv3(16->16);
 *   head    conv1(16->4), no activation.
 *   conv3 = 3x3x3 convolution, zero padding 1, bias, ReLU; pool = 2x2x2
 *   average; up = 2x nearest-neighbour upsampling; concat puts the upsampled
 *   channels first.  354,628 parameters.
 *
 * Parameter vector (FP32, host or device order identical): for each of the 11
 * convolutions in the order above, weights [co][ci][kz][ky][kx] followed by
 * bias [co].  The forward and backward passes use the weights rounded to
 * BF16 (round to nearest even) and FP32 arithmetic; Adam updates the FP32
 * master copy.
 *
 * Tensors: FP32 device arrays [batch][channel][z][y][x] (x fastest),
 * r = res cells per axis.  Every pointer argument named *_dev is a device
 * pointer the caller owns; *_host arguments are host memory.  All work is
 * enqueued on the stream given at creation; calls that return host values
 * synchronize with it.  Errors: return codes below; nothing throws;
 * kvnn_last_error() describes the last failure of a handle.
 */
#ifndef KVNN_H
#define KVNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kvnn kvnn;

enum { KVNN_OK = 0, KVNN_EINVAL = 1, KVNN_ENOMEM = 2, KVNN_EDEVICE = 3 };

typedef struct {
  int res;                      /* cells per axis, a multiple of 4, 4..256 */
  int batch_max;                /* largest batch of any later call, >= 1 */
  const double *xc, *yc, *zc;   /* host, res cell-centre coordinates each, in [0,1] */
  double lgr_lo, lgr_hi;        /* log10 Gr range mapped to [-1, 1]; lgr_hi > lgr_lo */
  uint64_t seed;                /* He-normal initial weights, zero biases */
} kvnn_params;

/* Creates a network and its device buffers (activations for batch_max). */
int kvnn_create(const kvnn_params* p, void* hip_stream, kvnn** out);
/* Frees everything; a null handle is accepted. */
int kvnn_destroy(kvnn* net);
/* Number of parameters (FP32 values). */
int kvnn_num_params(const kvnn* net, int64_t* count);
/* Copies the FP32 master parameters to host memory (count values). */
int kvnn_get_params(kvnn* net, float* params_host);
/* Replaces the master parameters and resets the Adam state and step count. */
int kvnn_set_params(kvnn* net, const float* params_host);
/* Builds the 4 input channels for batch Gr values (host array) into
 * in_dev [batch][4][r][r][r].  Gr > 0. */
int kvnn_make_inputs(kvnn* net, const double* gr_host, int batch, float* in_dev);
/* Forward pass: out_dev [batch][4][r][r][r] (may be null: the result stays
 * in the handle's buffer). */
int kvnn_forward(kvnn* net, const float* in_dev, int batch, float* out_dev);
/* kvnn_make_inputs for one Gr followed by kvnn_forward. */
int kvnn_predict(kvnn* net, double Gr, float* out_dev);
/* Gradient of sum(out * gout_dev) with respect to the parameters, through
 * the BF16-rounded weights (a forward pass is run first).  grads_host: count
 * FP32 values, may be null (gradients stay on the device). */
int kvnn_backward(kvnn* net, const float* in_dev, const float* gout_dev, int batch, float* grads_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean squared error mean((out - target)^2) over all batch*4*r^3 values.
 * loss_host (nullable) receives the loss before the step. */
int kvnn_train_step(kvnn* net, const float* in_dev, const float* target_dev, int batch, float lr,
                    float* loss_host);
/* Message of the last failure on this handle. */
const char* kvnn_last_error(const kvnn* net);

#ifdef __cplusplus
}
#endif

#endif /* KVNN_H */
