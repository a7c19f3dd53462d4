// Device helpers for the gfx950 kernels: complex arithmetic, storage formats,
// neighbour indexing, block reductions and the XCD-aware block order.
#pragma once

#include "stag_internal.h"

namespace stag {

template <int P> struct RealOf { using T = float; };
template <> struct RealOf<P64> { using T = double; };

template <typename T> struct Cx { T re, im; };

template <typename T> __device__ __forceinline__ void cmac(Cx<T>& acc, const Cx<T>& a, const Cx<T>& b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

// acc += U v  (U row-major: element 3a+b)
template <typename T> __device__ __forceinline__ void matvec_acc(const Cx<T> u[9], const Cx<T> v[3], Cx<T> acc[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) cmac(acc[a], u[3 * a + b], v[b]);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block i -> XCD i % 8).
// Renumber them so that each XCD walks one contiguous range of tiles: neighbour
// colour vectors then stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// ---- binary16 helpers -------------------------------------------------------
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Cx<float> unpack_h2(unsigned w, float s) {
  h2v h = __builtin_bit_cast(h2v, w);
  return Cx<float>{(float)h.x * s, (float)h.y * s};
}
__device__ __forceinline__ unsigned pack_h2(float a, float b) {
  h2v h;
  h.x = (_Float16)a;
  h.y = (_Float16)b;
  return __builtin_bit_cast(unsigned, h);
}

// ---- colour vectors ---------------------------------------------------------
// f64: 3 x double2 (48 B); f32: 3 x float2 (24 B); f16: uint4 = 6 binary16 codes + binary32 scale (16 B).
template <int P> __device__ __forceinline__ void load_spinor(const void* base, long s, Cx<typename RealOf<P>::T> v[3]);

template <> __device__ __forceinline__ void load_spinor<P64>(const void* base, long s, Cx<double> v[3]) {
  const double2* p = reinterpret_cast<const double2*>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double2 w = p[c];
    v[c] = Cx<double>{w.x, w.y};
  }
}
template <> __device__ __forceinline__ void load_spinor<P32>(const void* base, long s, Cx<float> v[3]) {
  const float2* p = reinterpret_cast<const float2*>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float2 w = p[c];
    v[c] = Cx<float>{w.x, w.y};
  }
}
template <> __device__ __forceinline__ void load_spinor<P16>(const void* base, long s, Cx<float> v[3]) {
  const uint4 w = reinterpret_cast<const uint4*>(base)[s];
  const float sc = __uint_as_float(w.w);
  v[0] = unpack_h2(w.x, sc);
  v[1] = unpack_h2(w.y, sc);
  v[2] = unpack_h2(w.z, sc);
}

// Store and return the stored (rounded) value in v.
template <int P> __device__ __forceinline__ void store_spinor(void* base, long s, Cx<typename RealOf<P>::T> v[3]);

template <> __device__ __forceinline__ void store_spinor<P64>(void* base, long s, Cx<double> v[3]) {
  double2* p = reinterpret_cast<double2*>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = make_double2(v[c].re, v[c].im);
}
template <> __device__ __forceinline__ void store_spinor<P32>(void* base, long s, Cx<float> v[3]) {
  float2* p = reinterpret_cast<float2*>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = make_float2(v[c].re, v[c].im);
}
template <> __device__ __forceinline__ void store_spinor<P16>(void* base, long s, Cx<float> v[3]) {
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
  uint4 w;
  if (m > 0.f) {
    w.x = pack_h2(v[0].re / m, v[0].im / m);
    w.y = pack_h2(v[1].re / m, v[1].im / m);
    w.z = pack_h2(v[2].re / m, v[2].im / m);
  } else {
    w.x = w.y = w.z = 0u;
  }
  w.w = __float_as_uint(m);
  reinterpret_cast<uint4*>(base)[s] = w;
  v[0] = unpack_h2(w.x, m);
  v[1] = unpack_h2(w.y, m);
  v[2] = unpack_h2(w.z, m);
}

// ---- packed links -----------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

// Links for one output parity are stored per block of 64 output sites and per
// link k as 16-byte chunks: chunk j of (block, k) holds, for the 64 lanes in
// order, the j-th 16-byte piece of each lane's 9 complex numbers.  A wave's
// load of one chunk is therefore one contiguous 1 KiB (the tail chunk is
// narrower).  Byte offset of (block, k): (block * 16 + k) * 64 * link_bytes(P).
template <int P> __device__ __forceinline__ void load_link(const char* base, long blk, int k, int lane,
                                                           float scale, Cx<typename RealOf<P>::T> u[9]);

template <> __device__ __forceinline__ void load_link<P64>(const char* base, long blk, int k, int lane, float,
                                                           Cx<double> u[9]) {
  const d2v* p = reinterpret_cast<const d2v*>(base + (blk * kLinks + k) * (long)(kWave * 144)) + lane;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    d2v w = __builtin_nontemporal_load(p + e * kWave);
    u[e] = Cx<double>{w.x, w.y};
  }
}
template <> __device__ __forceinline__ void load_link<P32>(const char* base, long blk, int k, int lane, float,
                                                           Cx<float> u[9]) {
  const char* b = base + (blk * kLinks + k) * (long)(kWave * 72);
  const f4v* p = reinterpret_cast<const f4v*>(b) + lane;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    f4v w = __builtin_nontemporal_load(p + j * kWave);
    u[2 * j] = Cx<float>{w.x, w.y};
    u[2 * j + 1] = Cx<float>{w.z, w.w};
  }
  f2v w = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(b + 4 * kWave * 16) + lane);
  u[8] = Cx<float>{w.x, w.y};
}
template <> __device__ __forceinline__ void load_link<P16>(const char* base, long blk, int k, int lane, float s,
                                                           Cx<float> u[9]) {
  const char* b = base + (blk * kLinks + k) * (long)(kWave * 36);
  const u4v* p = reinterpret_cast<const u4v*>(b) + lane;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    u4v w = __builtin_nontemporal_load(p + j * kWave);
    u[4 * j + 0] = unpack_h2(w.x, s);
    u[4 * j + 1] = unpack_h2(w.y, s);
    u[4 * j + 2] = unpack_h2(w.z, s);
    u[4 * j + 3] = unpack_h2(w.w, s);
  }
  unsigned w = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(b + 2 * kWave * 16) + lane);
  u[8] = unpack_h2(w, s);
}

// ---- geometry -----------------------------------------------------------------
struct Site {
  int cb, x, y, z, t;
};

__device__ __forceinline__ Site site_of(int cb, int par, const Geo& g) {
  Site s;
  s.cb = cb;
  int xh = cb % g.Xh;
  int rest = cb / g.Xh;
  s.y = rest % g.L[1];
  rest /= g.L[1];
  s.z = rest % g.L[2];
  s.t = rest / g.L[2];
  s.x = 2 * xh + ((s.y + s.z + s.t + par) & 1);
  return s;
}

__device__ __forceinline__ int wrap_fwd(int v, int h, int L) { v += h; return v >= L ? v - L : v; }
__device__ __forceinline__ int wrap_bwd(int v, int h, int L) { v -= h; return v < 0 ? v + L : v; }

// cb of the neighbour n +- h mu (h already reduced mod L_mu); branch-free selects.
__device__ __forceinline__ int neighbour(const Site& s, const Geo& g, int mu, int h, bool fwd) {
  if (mu == 0) {
    int xn = fwd ? wrap_fwd(s.x, h, g.L[0]) : wrap_bwd(s.x, h, g.L[0]);
    return s.cb - (s.x >> 1) + (xn >> 1);
  }
  int c = mu == 1 ? s.y : (mu == 2 ? s.z : s.t);
  int cn = fwd ? wrap_fwd(c, h, g.L[mu]) : wrap_bwd(c, h, g.L[mu]);
  return s.cb + (cn - c) * g.stride[mu];
}

// ---- reductions ---------------------------------------------------------------
// Deterministic block sum of N doubles per thread; the result is valid in thread 0.
template <int N> __device__ __forceinline__ void block_sum(double v[N], double* lds /* >= N * 4 */) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, kWave);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (nw == 1) return;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) lds[i * 4 + wave] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = lds[i * 4];
      for (int w = 1; w < nw; ++w) s += lds[i * 4 + w];
      v[i] = s;
    }
}

__device__ __forceinline__ int find_problem(const Batch& B, int bid) {
  int p = 0;
#pragma unroll 1
  while (p + 1 < B.nprob && bid >= B.block_start[p + 1]) ++p;
  return p;
}

// gate: 0 = every slot not finished (state <= 2), 1 = running (state 0),
//       2 = running or pending x update (state <= 1), 3 = every slot, 4 = state 1 only
__device__ __forceinline__ bool slot_on(const Scal* scal, int slot, int gate) {
  if (gate == 3) return true;
  const int st = scal[slot].state;
  switch (gate) {
    case 1: return st == 0;
    case 2: return st <= 1;
    case 4: return st == 1;
    default: return st <= 2;
  }
}

}  // namespace stag
