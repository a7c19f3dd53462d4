// Link ingest and packing, and colour-vector precision conversions.
//
// Packing folds into each of the 16 matrices an output site uses (Sec. 2, Eq. (5):
// the staggered phases are absorbed into the stored links):
//   k = 4 mu + 0 : eta_mu(n) s(n,1) F_mu(n)                       (neighbour n + mu)
//   k = 4 mu + 1 : -eta_mu(n) s(n-mu,1) F_mu(n-mu)^dag            (neighbour n - mu)
//   k = 4 mu + 2 : c_N eta_mu(n) s(n,3) W_mu(n)                   (neighbour n + 3mu)
//   k = 4 mu + 3 : -c_N eta_mu(n) s(n-3mu,3) W_mu(n-3mu)^dag      (neighbour n - 3mu)
// with s(m,k) = (-1)^floor((m_t + k)/L_t) for the time direction when it is
// antiperiodic and 1 otherwise.  Back links are duplicated per output parity so
// the Dslash streams exactly 16 matrices per site, coalesced (Sec. 3.1).
#include "device.h"
#include "launch.h"

namespace stag {

Geo make_geo(const int dims[4]) {
  Geo g{};
  for (int i = 0; i < 4; ++i) {
    g.L[i] = dims[i];
    g.h1[i] = 1 % dims[i];
    g.h3[i] = 3 % dims[i];
  }
  g.Xh = dims[0] / 2;
  g.half = (int)((long)dims[0] * dims[1] * dims[2] * dims[3] / 2);
  g.stride[0] = 0;
  g.stride[1] = g.Xh;
  g.stride[2] = g.Xh * dims[1];
  g.stride[3] = g.Xh * dims[1] * dims[2];
  g.t0 = 0;
  g.lt_glob = dims[3];
  g.h3g = 3 % dims[3];
  g.t_open = 0;
  g.in_half = g.half;
  return g;
}

// Folded matrix k at output site s (FP64).
__device__ void folded_link(const double2* fat, const double2* lng, double naik, const Geo& g, int antiper,
                            const Site& s, int k, double2 u[9]) {
  const int mu = k >> 2, j = k & 3;
  const bool is_long = j >= 2, bwd = (j & 1) != 0;
  const int hop = is_long ? 3 : 1;
  const double2* src = is_long ? lng : fat;
  if (src == nullptr) {
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = make_double2(0.0, 0.0);
    return;
  }
  int c[4] = {s.x, s.y, s.z, s.t};
  const int eta_sum = (mu > 0 ? c[0] : 0) + (mu > 1 ? c[1] : 0) + (mu > 2 ? c[2] : 0);
  double coef = (eta_sum & 1) ? -1.0 : 1.0;
  if (is_long) coef *= naik;
  if (bwd) {
    c[mu] = ((c[mu] - hop) % g.L[mu] + g.L[mu]) % g.L[mu];  // start site m = n - hop mu
    coef = -coef;
  }
  if (mu == 3 && antiper && (((c[3] + hop) / g.L[3]) & 1)) coef = -coef;
  const long site = (((long)c[3] * g.L[2] + c[2]) * g.L[1] + c[1]) * g.L[0] + c[0];
  const long vol = (long)g.half * 2;
  const double2* U = src + ((long)mu * vol + site) * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      // forward: U[a][b]; backward: (U^dag)[a][b] = conj(U[b][a])
      const double2 w = bwd ? U[3 * b + a] : U[3 * a + b];
      u[3 * a + b] = make_double2(coef * w.x, bwd ? -coef * w.y : coef * w.y);
    }
}

// binary16 code of v / s with the quotient rounded first to binary32 (both round-to-nearest-even).
__device__ __forceinline__ _Float16 f16_code(double v, float s) {
  return s > 0.f ? (_Float16)(float)(v / (double)s) : (_Float16)0.f;
}

template <int P>
__global__ __launch_bounds__(256) void k_pack_links(const double2* fat, const double2* lng, double naik, Geo g,
                                                    int antiper, int par, char* out, float* lscale) {
  const int cb_raw = blockIdx.x * blockDim.x + threadIdx.x;
  const int padded = ceil_div(g.half, kWave) * kWave;
  if (cb_raw >= padded) return;
  const bool live = cb_raw < g.half;
  const Site s = site_of(live ? cb_raw : 0, par, g);
  const long blk = cb_raw >> 6;
  const int lane = cb_raw & 63;
  float scale[2] = {0.f, 0.f};
  const bool c12 = g.long12 != 0;
  // FP64 with lscale: also compute the FP16 scales of the same matrices for k_pack_f16_from_f64, per
  // output site the largest |re|, |im| over the stored entries of its eight one-hop and, separately, its
  // eight three-hop matrices (rounded to binary32: the rounding of a max is the max of the roundings)
  const bool scales64 = P == P64 && lscale != nullptr;
  for (int k = 0; k < kLinks; ++k) {
    double2 u[9];
    if (live) {
      folded_link(fat, lng, naik, g, antiper, s, k, u);
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = make_double2(0.0, 0.0);
    }
    char* base = out + link_slot_offset(P, c12, blk, k);
    const bool two_rows = c12 && ((k & 3) >= 2);
    if (P == P64) {
      double2* o = reinterpret_cast<double2*>(base) + lane;
#pragma unroll
      for (int e = 0; e < 9; ++e)
        if (e < (two_rows ? 6 : 9)) o[e * kWave] = u[e];
      if (scales64 && live) {
        double m = 0.0;
#pragma unroll
        for (int e = 0; e < 9; ++e)
          if (e < (two_rows ? 6 : 9)) m = fmax(m, fmax(fabs(u[e].x), fabs(u[e].y)));
        scale[(k >> 1) & 1] = fmaxf(scale[(k >> 1) & 1], (float)m);
      }
    } else {
      static_assert(P == P64 || P == P32, "FP16 is packed from the FP64 matrices (k_pack_f16_from_f64)");
      float4* o = reinterpret_cast<float4*>(base) + lane;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < (two_rows ? 3 : 4))
          o[j * kWave] = make_float4((float)u[2 * j].x, (float)u[2 * j].y, (float)u[2 * j + 1].x, (float)u[2 * j + 1].y);
      if (!two_rows) reinterpret_cast<float2*>(base + 4 * kWave * 16)[lane] = make_float2((float)u[8].x, (float)u[8].y);
    }
  }
  if (scales64) {
    lscale[blk * 2 * kWave + lane] = scale[0];
    lscale[blk * 2 * kWave + kWave + lane] = scale[1];
  }
}

// FP16 packing from the FP64 packed matrices and the scales the FP64 pack computed (when both are
// requested): one coalesced pass over the packed FP64 blocks instead of folding every link again from
// the input fields twice (once for the scales, once for the codes).  The codes are the same, since the
// FP64 packed entries are the folded matrices themselves.
__global__ __launch_bounds__(256) void k_pack_f16_from_f64(const char* packed64, const float* lscale, int half,
                                                          int c12, char* out) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const int padded = ceil_div(half, kWave) * kWave;
  if (cb >= padded) return;
  const long blk = cb >> 6;
  const int lane = cb & 63;
  const float scale[2] = {lscale[blk * 2 * kWave + lane], lscale[blk * 2 * kWave + kWave + lane]};
  for (int k = 0; k < kLinks; ++k) {
    const bool two_rows = c12 && ((k & 3) >= 2);
    const double2* in = reinterpret_cast<const double2*>(packed64 + link_slot_offset(P64, c12, blk, k)) + lane;
    double2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = e < (two_rows ? 6 : 9) ? in[e * kWave] : make_double2(0.0, 0.0);
    const float sc = scale[(k >> 1) & 1];
    h2v h[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      h[e].x = f16_code(u[e].x, sc);
      h[e].y = f16_code(u[e].y, sc);
    }
    char* base = out + link_slot_offset(P16, c12, blk, k);
    uint4* o = reinterpret_cast<uint4*>(base) + lane;
    if (two_rows) {
      o[0] = make_uint4(__builtin_bit_cast(unsigned, h[0]), __builtin_bit_cast(unsigned, h[1]),
                        __builtin_bit_cast(unsigned, h[2]), __builtin_bit_cast(unsigned, h[3]));
      reinterpret_cast<uint2*>(base + kWave * 16)[lane] =
          make_uint2(__builtin_bit_cast(unsigned, h[4]), __builtin_bit_cast(unsigned, h[5]));
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j)
        o[j * kWave] = make_uint4(__builtin_bit_cast(unsigned, h[4 * j]), __builtin_bit_cast(unsigned, h[4 * j + 1]),
                                  __builtin_bit_cast(unsigned, h[4 * j + 2]), __builtin_bit_cast(unsigned, h[4 * j + 3]));
      reinterpret_cast<unsigned*>(base + 2 * kWave * 16)[lane] = __builtin_bit_cast(unsigned, h[8]);
    }
  }
}

hipError_t launch_pack_f16_from_f64(const void* packed64, const float* lscale, const Geo& g, void* out,
                                    hipStream_t st) {
  const int padded = ceil_div(g.half, kWave) * kWave;
  k_pack_f16_from_f64<<<ceil_div(padded, 256), 256, 0, st>>>(reinterpret_cast<const char*>(packed64), lscale, g.half,
                                                             g.long12, reinterpret_cast<char*>(out));
  return hipGetLastError();
}

hipError_t launch_pack_links(int prec, const void* fat, const void* lng, double naik, const Geo& g, int antiper,
                             int par, void* out, float* lscale, hipStream_t st) {
  const int padded = ceil_div(g.half, kWave) * kWave;
  const int nblk = ceil_div(padded, 256);
  auto f = reinterpret_cast<const double2*>(fat);
  auto l = reinterpret_cast<const double2*>(lng);
  auto o = reinterpret_cast<char*>(out);
  switch (prec) {
    case P64: k_pack_links<P64><<<nblk, 256, 0, st>>>(f, l, naik, g, antiper, par, o, lscale); break;
    case P32: k_pack_links<P32><<<nblk, 256, 0, st>>>(f, l, naik, g, antiper, par, o, lscale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- colour-vector conversions ---------------------------------------------------
// complex128 -> storage format; f16 uses the per-site rule s = binary32(max |v|),
// code = binary16(binary32(v / s)).
template <int P>
__global__ __launch_bounds__(256) void k_from_f64(const double2* in, char* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2* v = in + 3 * i;
  double2 w[3] = {v[0], v[1], v[2]};
  if (P == P32) {
    float2* o = reinterpret_cast<float2*>(out) + 3 * i;
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = make_float2((float)w[c].x, (float)w[c].y);
  } else if (P == P16) {
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) m = fmax(m, fmax(fabs(w[c].x), fabs(w[c].y)));
    const float s = (float)m;
    h2v h[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h[c].x = f16_code(w[c].x, s);
      h[c].y = f16_code(w[c].y, s);
    }
    reinterpret_cast<uint4*>(out)[i] = make_uint4(__builtin_bit_cast(unsigned, h[0]), __builtin_bit_cast(unsigned, h[1]),
                                                  __builtin_bit_cast(unsigned, h[2]), __float_as_uint(s));
  } else {
    double2* o = reinterpret_cast<double2*>(out) + 3 * i;
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = w[c];
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_to_f64(const char* in, double2* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Cx<typename RealOf<P>::T> v[3];
  load_spinor<P>(in, i, v);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[3 * i + c] = make_double2((double)v[c].re, (double)v[c].im);
}

hipError_t launch_convert_from_f64(int prec, const void* in, void* out, long nsites, hipStream_t st) {
  if (nsites == 0) return hipSuccess;
  const long nblk = (nsites + 255) / 256;
  auto i = reinterpret_cast<const double2*>(in);
  auto o = reinterpret_cast<char*>(out);
  switch (prec) {
    case P64: k_from_f64<P64><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    case P32: k_from_f64<P32><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    case P16: k_from_f64<P16><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_convert_to_f64(int prec, const void* in, void* out, long nsites, hipStream_t st) {
  if (nsites == 0) return hipSuccess;
  const long nblk = (nsites + 255) / 256;
  auto i = reinterpret_cast<const char*>(in);
  auto o = reinterpret_cast<double2*>(out);
  switch (prec) {
    case P64: k_to_f64<P64><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    case P32: k_to_f64<P32><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    case P16: k_to_f64<P16><<<nblk, 256, 0, st>>>(i, o, nsites); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace stag
