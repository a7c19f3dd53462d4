// Launch interface of the network kernels (net.hip).
#pragma once

#include "stag_internal.h"

namespace stag {

struct NetLayerArgs {
  Geo g;
  const char* links;       // packed FP32 links for output parity out_par
  int out_par;
  const float2* in_same;   // [CIN][V/2][3] on parity out_par, or null (zero field)
  const float2* in_other;  // [CIN][V/2][3] on parity 1 - out_par, or null (zero field)
  float2* out;             // [COUT][V/2][3] on parity out_par
  const float2* w;         // [9][COUT][CIN] complex64 weights of the layer
};

hipError_t launch_net_layer(const NetLayerArgs& a, int cin, int cout, hipStream_t st);
hipError_t launch_net_wgrad(const NetLayerArgs& a, const float2* gy, double* partial, int cin, int cout, int nblk,
                            hipStream_t st);
hipError_t launch_net_wgrad_reduce(const double* partial, int cin, int cout, int nblk, int npar, double* out,
                                   hipStream_t st);
hipError_t launch_net_embed(const void* in, float2* out, long nsites, hipStream_t st);
hipError_t launch_net_extract(const float2* in, void* out, long nsites, hipStream_t st);
hipError_t launch_net_loss(const float2* out, const void* x, double scale, float2* g, double* partial, double* sum,
                           long nsites, hipStream_t st);
hipError_t launch_norm2_c128(const void* x, double* partial, double* sum, long nsites, hipStream_t st);
hipError_t launch_sub_norm(const void* a, const void* b, void* out, double* partial, double* sum, long nsites,
                           hipStream_t st);
hipError_t launch_scale_to_f32(const void* in, double scale, float2* out, long nsites, hipStream_t st);

}  // namespace stag
