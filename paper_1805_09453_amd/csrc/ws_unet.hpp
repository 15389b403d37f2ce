// Internal interface of the warm-start network (ws_unet.hip) used by the C ABI
// in gprox.hip.  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

struct ws_net;

namespace wsi {

// Network with activations for up to max_batch inputs of ny x nx (multiples of 8).
int create(ws_net** out, int max_batch, int ny, int nx, char* err, size_t errlen);
void destroy(ws_net* net);
long long param_count();
void native(const ws_net* net, int* ny, int* nx, int* max_batch);
const char* error(const ws_net* net);

// FP32 parameter blob (device pointers, layout in include/gprox.h); set resets Adam.
int set_params(ws_net* net, hipStream_t s, const float* blob);
int get_params(ws_net* net, hipStream_t s, float* blob);

// phi = net(rho0, rho1) for `batch` inputs at the native size, FP32 [batch][ny][nx].
int predict(ws_net* net, hipStream_t s, const float* rho0, const float* rho1, int batch, float* phi);

// Loss against phi_star (mean squared grad_h error, h the target's spacing) and the
// parameter gradients into the net's gradient blob (copied to grad_out if non-null).
// Synchronises s to return the loss.
int grads(ws_net* net, hipStream_t s, const float* rho0, const float* rho1, const float* phi_star, int batch,
          double h, float* grad_out, double* loss);

// One Adam step with the gradients of the last grads() call.
int adam(ws_net* net, hipStream_t s, double lr);

// f x f block mean (FP32 [ny][nx] -> [ny/f][nx/f]) and cell-centred bilinear
// interpolation ([ny][nx] -> [f ny][f nx]).
int downsample(hipStream_t s, const float* in, int ny, int nx, int f, float* out);
int upsample(hipStream_t s, const float* in, int ny, int nx, int f, float* out);

}  // namespace wsi
