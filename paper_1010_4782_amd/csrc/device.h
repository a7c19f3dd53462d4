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

// ---- global-memory pointers -----------------------------------------------------
// Buffers reach the kernels through structs in device memory, so the compiler cannot tell their
// address space and emits flat loads, which count against both vmcnt and lgkmcnt and force coarse
// waits.  Every buffer here is in global memory: casting to address space 1 gives global loads.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> using gptr_w = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(const void* p) { return (gptr<T>)p; }
template <typename T> __device__ __forceinline__ gptr_w<T> as_global_w(void* p) { return (gptr_w<T>)p; }

// ---- colour vectors ---------------------------------------------------------
// f64: 3 x double2 (48 B); f32: 3 x float2 (24 B); f16: uint4 = 6 binary16 codes + binary32 scale (16 B).
// NT = true: a non-temporal access, for vectors a kernel streams once (the vector updates of CG);
// vectors that are read again (the Dslash's neighbours) use the default, which keeps them in L2.
template <typename V, bool NT> __device__ __forceinline__ V ld(gptr<V> p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename V, bool NT> __device__ __forceinline__ void st(gptr_w<V> p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <int P, bool NT = false>
__device__ __forceinline__ void load_spinor(const void* base, long s, Cx<typename RealOf<P>::T> v[3]) {
  if constexpr (P == P64) {
    gptr<d2v> p = as_global<d2v>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const d2v w = ld<d2v, NT>(p + c);
      v[c] = Cx<double>{w.x, w.y};
    }
  } else if constexpr (P == P32) {
    gptr<f2v> p = as_global<f2v>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const f2v w = ld<f2v, NT>(p + c);
      v[c] = Cx<float>{w.x, w.y};
    }
  } else {
    const u4v w = ld<u4v, NT>(as_global<u4v>(base) + s);
    const float sc = __uint_as_float(w.w);
    v[0] = unpack_h2(w.x, sc);
    v[1] = unpack_h2(w.y, sc);
    v[2] = unpack_h2(w.z, sc);
  }
}

// Colour-vector loads for the Dslash, which keeps FP16 link matrices in code units and folds the
// link's scale into the vector instead: v = (link scale x vector scale) x codes, one multiply per
// component instead of one per matrix element.  For FP32 and FP64 (no scales) these are the plain loads.
template <int P>
__device__ __forceinline__ void load_spinor_ls(const void* base, long s, float lsc, Cx<typename RealOf<P>::T> v[3]) {
  if constexpr (P == P16) {
    const u4v w = as_global<u4v>(base)[s];
    const float sc = __uint_as_float(w.w) * lsc;
    v[0] = unpack_h2(w.x, sc);
    v[1] = unpack_h2(w.y, sc);
    v[2] = unpack_h2(w.z, sc);
  } else {
    load_spinor<P>(base, s, v);
  }
}

// The same reads from a colour-vector array staged in LDS (index s relative to the staged window).
template <int P>
__device__ __forceinline__ void load_spinor_lds(const char* base, int s, float lsc, Cx<typename RealOf<P>::T> v[3]) {
  if constexpr (P == P64) {
    const d2v* p = reinterpret_cast<const d2v*>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = Cx<double>{p[c].x, p[c].y};
  } else if constexpr (P == P32) {
    const f2v* p = reinterpret_cast<const f2v*>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = Cx<float>{p[c].x, p[c].y};
  } else {
    const u4v w = reinterpret_cast<const u4v*>(base)[s];
    const float sc = __uint_as_float(w.w) * lsc;
    v[0] = unpack_h2(w.x, sc);
    v[1] = unpack_h2(w.y, sc);
    v[2] = unpack_h2(w.z, sc);
  }
}

// Store and return the stored (rounded) value in v.  FP16: code = binary16(v / m), m = max |component|;
// RCP takes the six quotients as v x binary32(1 / m), one division per site instead of six (each
// quotient then within 2^-23 of v / m, far below the binary16 rounding that follows): the Dslash
// epilogues, where the divisions are a tenth of the arithmetic.  A subnormal m (the edge of a point
// source's spreading support reaches 1e-39) keeps the six divisions: 1 / m would overflow.
template <int P, bool NT = false, bool RCP = false>
__device__ __forceinline__ void store_spinor(void* base, long s, Cx<typename RealOf<P>::T> v[3]) {
  if constexpr (P == P64) {
    gptr_w<d2v> p = as_global_w<d2v>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) st<d2v, NT>(p + c, d2v{v[c].re, v[c].im});
  } else if constexpr (P == P32) {
    gptr_w<f2v> p = as_global_w<f2v>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) st<f2v, NT>(p + c, f2v{v[c].re, v[c].im});
  } else {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    unsigned w0 = 0u, w1 = 0u, w2 = 0u;
    if (m > 0.f) {
      if (RCP && m >= 0x1p-126f) {
        const float inv = 1.f / m;
        w0 = pack_h2(v[0].re * inv, v[0].im * inv);
        w1 = pack_h2(v[1].re * inv, v[1].im * inv);
        w2 = pack_h2(v[2].re * inv, v[2].im * inv);
      } else {
        w0 = pack_h2(v[0].re / m, v[0].im / m);
        w1 = pack_h2(v[1].re / m, v[1].im / m);
        w2 = pack_h2(v[2].re / m, v[2].im / m);
      }
    }
    st<u4v, NT>(as_global_w<u4v>(base) + s, u4v{w0, w1, w2, __float_as_uint(m)});
    v[0] = unpack_h2(w0, m);
    v[1] = unpack_h2(w1, m);
    v[2] = unpack_h2(w2, m);
  }
}

// ---- packed links -----------------------------------------------------------
// A slot holds, for the 64 lanes of a block, each lane's link as 16-byte chunks: chunk j of all 64
// lanes is contiguous (one wave load = 1 KiB), and a narrower tail chunk follows the full ones.
// rows = 3 loads the whole matrix, rows = 2 the first two rows of a compressed three-hop link.

template <int P, int ROWS>
__device__ __forceinline__ void load_link_rows(const char* slot, int lane, float scale, Cx<typename RealOf<P>::T> u[9]);

template <> __device__ __forceinline__ void load_link_rows<P64, 3>(const char* slot, int lane, float, Cx<double> u[9]) {
  gptr<d2v> p = as_global<d2v>(slot) + lane;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    d2v w = __builtin_nontemporal_load(p + e * kWave);
    u[e] = Cx<double>{w.x, w.y};
  }
}
template <> __device__ __forceinline__ void load_link_rows<P64, 2>(const char* slot, int lane, float, Cx<double> u[9]) {
  gptr<d2v> p = as_global<d2v>(slot) + lane;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    d2v w = __builtin_nontemporal_load(p + e * kWave);
    u[e] = Cx<double>{w.x, w.y};
  }
}
template <> __device__ __forceinline__ void load_link_rows<P32, 3>(const char* slot, int lane, float, Cx<float> u[9]) {
  gptr<f4v> p = as_global<f4v>(slot) + lane;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    f4v w = __builtin_nontemporal_load(p + j * kWave);
    u[2 * j] = Cx<float>{w.x, w.y};
    u[2 * j + 1] = Cx<float>{w.z, w.w};
  }
  f2v w = __builtin_nontemporal_load(as_global<f2v>(slot + 4 * kWave * 16) + lane);
  u[8] = Cx<float>{w.x, w.y};
}
template <> __device__ __forceinline__ void load_link_rows<P32, 2>(const char* slot, int lane, float, Cx<float> u[9]) {
  gptr<f4v> p = as_global<f4v>(slot) + lane;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    f4v w = __builtin_nontemporal_load(p + j * kWave);
    u[2 * j] = Cx<float>{w.x, w.y};
    u[2 * j + 1] = Cx<float>{w.z, w.w};
  }
}
template <> __device__ __forceinline__ void load_link_rows<P16, 3>(const char* slot, int lane, float s, Cx<float> u[9]) {
  gptr<u4v> p = as_global<u4v>(slot) + lane;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    u4v w = __builtin_nontemporal_load(p + j * kWave);
    u[4 * j + 0] = unpack_h2(w.x, s);
    u[4 * j + 1] = unpack_h2(w.y, s);
    u[4 * j + 2] = unpack_h2(w.z, s);
    u[4 * j + 3] = unpack_h2(w.w, s);
  }
  unsigned w = __builtin_nontemporal_load(as_global<unsigned>(slot + 2 * kWave * 16) + lane);
  u[8] = unpack_h2(w, s);
}
template <> __device__ __forceinline__ void load_link_rows<P16, 2>(const char* slot, int lane, float s, Cx<float> u[9]) {
  u4v w = __builtin_nontemporal_load(as_global<u4v>(slot) + lane);
  u[0] = unpack_h2(w.x, s);
  u[1] = unpack_h2(w.y, s);
  u[2] = unpack_h2(w.z, s);
  u[3] = unpack_h2(w.w, s);
  u2v t = __builtin_nontemporal_load(as_global<u2v>(slot + kWave * 16) + lane);
  u[4] = unpack_h2(t.x, s);
  u[5] = unpack_h2(t.y, s);
}

// ---- raw (undecoded) loads for software-pipelined kernels ---------------------------------
// The loaded registers are decoded only where they are used, so a load issued several links
// ahead is not waited for until then.
template <int P> struct RawLink;
template <> struct RawLink<P64> { d2v e[9]; };
template <> struct RawLink<P32> { f4v q[4]; f2v t; };
template <> struct RawLink<P16> { u4v q0, q1; unsigned t; };

template <int P, int ROWS> __device__ __forceinline__ void raw_link_load(const char* slot, int lane, RawLink<P>& r);
template <> __device__ __forceinline__ void raw_link_load<P64, 3>(const char* slot, int lane, RawLink<P64>& r) {
  gptr<d2v> p = as_global<d2v>(slot) + lane;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.e[e] = __builtin_nontemporal_load(p + e * kWave);
}
template <> __device__ __forceinline__ void raw_link_load<P64, 2>(const char* slot, int lane, RawLink<P64>& r) {
  gptr<d2v> p = as_global<d2v>(slot) + lane;
#pragma unroll
  for (int e = 0; e < 6; ++e) r.e[e] = __builtin_nontemporal_load(p + e * kWave);
}
template <> __device__ __forceinline__ void raw_link_load<P32, 3>(const char* slot, int lane, RawLink<P32>& r) {
  gptr<f4v> p = as_global<f4v>(slot) + lane;
#pragma unroll
  for (int j = 0; j < 4; ++j) r.q[j] = __builtin_nontemporal_load(p + j * kWave);
  r.t = __builtin_nontemporal_load(as_global<f2v>(slot + 4 * kWave * 16) + lane);
}
template <> __device__ __forceinline__ void raw_link_load<P32, 2>(const char* slot, int lane, RawLink<P32>& r) {
  gptr<f4v> p = as_global<f4v>(slot) + lane;
#pragma unroll
  for (int j = 0; j < 3; ++j) r.q[j] = __builtin_nontemporal_load(p + j * kWave);
}
template <> __device__ __forceinline__ void raw_link_load<P16, 3>(const char* slot, int lane, RawLink<P16>& r) {
  gptr<u4v> p = as_global<u4v>(slot) + lane;
  r.q0 = __builtin_nontemporal_load(p);
  r.q1 = __builtin_nontemporal_load(p + kWave);
  r.t = __builtin_nontemporal_load(as_global<unsigned>(slot + 2 * kWave * 16) + lane);
}
template <> __device__ __forceinline__ void raw_link_load<P16, 2>(const char* slot, int lane, RawLink<P16>& r) {
  r.q0 = __builtin_nontemporal_load(as_global<u4v>(slot) + lane);
  const u2v t = __builtin_nontemporal_load(as_global<u2v>(slot + kWave * 16) + lane);
  r.q1.x = t.x;
  r.q1.y = t.y;
}

template <int P, int ROWS>
__device__ __forceinline__ void raw_link_decode(const RawLink<P>& r, float scale, Cx<typename RealOf<P>::T> u[9]);
template <> __device__ __forceinline__ void raw_link_decode<P64, 3>(const RawLink<P64>& r, float, Cx<double> u[9]) {
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = Cx<double>{r.e[e].x, r.e[e].y};
}
template <> __device__ __forceinline__ void raw_link_decode<P64, 2>(const RawLink<P64>& r, float, Cx<double> u[9]) {
#pragma unroll
  for (int e = 0; e < 6; ++e) u[e] = Cx<double>{r.e[e].x, r.e[e].y};
}
template <> __device__ __forceinline__ void raw_link_decode<P32, 3>(const RawLink<P32>& r, float, Cx<float> u[9]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    u[2 * j] = Cx<float>{r.q[j].x, r.q[j].y};
    u[2 * j + 1] = Cx<float>{r.q[j].z, r.q[j].w};
  }
  u[8] = Cx<float>{r.t.x, r.t.y};
}
template <> __device__ __forceinline__ void raw_link_decode<P32, 2>(const RawLink<P32>& r, float, Cx<float> u[9]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    u[2 * j] = Cx<float>{r.q[j].x, r.q[j].y};
    u[2 * j + 1] = Cx<float>{r.q[j].z, r.q[j].w};
  }
}
template <> __device__ __forceinline__ void raw_link_decode<P16, 3>(const RawLink<P16>& r, float s, Cx<float> u[9]) {
  u[0] = unpack_h2(r.q0.x, s);
  u[1] = unpack_h2(r.q0.y, s);
  u[2] = unpack_h2(r.q0.z, s);
  u[3] = unpack_h2(r.q0.w, s);
  u[4] = unpack_h2(r.q1.x, s);
  u[5] = unpack_h2(r.q1.y, s);
  u[6] = unpack_h2(r.q1.z, s);
  u[7] = unpack_h2(r.q1.w, s);
  u[8] = unpack_h2(r.t, s);
}
template <> __device__ __forceinline__ void raw_link_decode<P16, 2>(const RawLink<P16>& r, float s, Cx<float> u[9]) {
  u[0] = unpack_h2(r.q0.x, s);
  u[1] = unpack_h2(r.q0.y, s);
  u[2] = unpack_h2(r.q0.z, s);
  u[3] = unpack_h2(r.q0.w, s);
  u[4] = unpack_h2(r.q1.x, s);
  u[5] = unpack_h2(r.q1.y, s);
}

template <int P> struct RawSpinor;
template <> struct RawSpinor<P64> { d2v c[3]; };
template <> struct RawSpinor<P32> { f2v c[3]; };
template <> struct RawSpinor<P16> { u4v w; };

template <int P> __device__ __forceinline__ void raw_spinor_load(const void* base, long s, RawSpinor<P>& r);
template <> __device__ __forceinline__ void raw_spinor_load<P64>(const void* base, long s, RawSpinor<P64>& r) {
  gptr<d2v> p = as_global<d2v>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) r.c[c] = p[c];
}
template <> __device__ __forceinline__ void raw_spinor_load<P32>(const void* base, long s, RawSpinor<P32>& r) {
  gptr<f2v> p = as_global<f2v>(base) + 3 * s;
#pragma unroll
  for (int c = 0; c < 3; ++c) r.c[c] = p[c];
}
template <> __device__ __forceinline__ void raw_spinor_load<P16>(const void* base, long s, RawSpinor<P16>& r) {
  r.w = as_global<u4v>(base)[s];
}
// The same raw reads from a colour-vector array staged in LDS (index s relative to the staged window).
template <int P> __device__ __forceinline__ void raw_spinor_lds(const char* base, int s, RawSpinor<P>& r) {
  if constexpr (P == P64) {
    const d2v* p = reinterpret_cast<const d2v*>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) r.c[c] = p[c];
  } else if constexpr (P == P32) {
    const f2v* p = reinterpret_cast<const f2v*>(base) + 3 * s;
#pragma unroll
    for (int c = 0; c < 3; ++c) r.c[c] = p[c];
  } else {
    r.w = reinterpret_cast<const u4v*>(base)[s];
  }
}
// lsc: the FP16 link scale folded into the vector (see load_spinor_ls); ignored for FP32 / FP64.
template <int P>
__device__ __forceinline__ void raw_spinor_decode(const RawSpinor<P>& r, float lsc, Cx<typename RealOf<P>::T> v[3]) {
  if constexpr (P == P16) {
    const float sc = __uint_as_float(r.w.w) * lsc;
    v[0] = unpack_h2(r.w.x, sc);
    v[1] = unpack_h2(r.w.y, sc);
    v[2] = unpack_h2(r.w.z, sc);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = {r.c[c].x, r.c[c].y};
  }
}

// Third row of s U for U in SU(3) from its first two rows a' = s a, b' = s b (paper Sec. 3.3,
// c = (a x b)^*):  s c = (a' x b')^* / s.
template <typename T>
__device__ __forceinline__ void rebuild_row3(Cx<T> u[9], T inv_s) {
  const Cx<T>* a = u;
  const Cx<T>* b = u + 3;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    // (a x b)_i = a_i1 b_i2 - a_i2 b_i1
    const T re = a[i1].re * b[i2].re - a[i1].im * b[i2].im - (a[i2].re * b[i1].re - a[i2].im * b[i1].im);
    const T im = a[i1].re * b[i2].im + a[i1].im * b[i2].re - (a[i2].re * b[i1].im + a[i2].im * b[i1].re);
    u[6 + i] = Cx<T>{re * inv_s, -im * inv_s};
  }
}

// ---- FP16 products on the binary16 codes (v_dot2_f32_f16) ----------------------------------------
// A binary16 link element u = (ur, ui) and colour component v = (vr, vi), each a pair of codes in one
// 32-bit word (real part in the low half):
//   Re(u v) = ur vr - ui vi = dot((ur, -ui), v),   Im(u v) = ui vr + ur vi = dot((ui, ur), v),
// two dot2 instructions per complex product, each multiplying two codes exactly and adding in binary32.
// The conjugated-sign word (ur, -ui) and the swapped word (ui, ur) are formed once per link element and
// serve every right-hand side.  The product of a link and a vector is taken in code units and then
// scaled by (link scale x vector scale).
__device__ __forceinline__ float fdot2(unsigned a, unsigned b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2v, a), __builtin_bit_cast(h2v, b), c, false);
}
__device__ __forceinline__ unsigned neg_hi(unsigned w) { return w ^ 0x80000000u; }                       // (a, b) -> (a, -b)
__device__ __forceinline__ unsigned swap_halves(unsigned w) { return __builtin_amdgcn_alignbit(w, w, 16); }  // (a, b) -> (b, a)

// A link in the dot2 form: its stored code words with the sign of the imaginary part flipped and with
// their halves swapped (9 each, or 6 for a two-row three-hop link), and, for a two-row link, its rebuilt
// third row in binary32 code units.
struct LinkH {
  unsigned p[9], s[9];
  Cx<float> w[3];
};

template <int ROWS>
__device__ __forceinline__ void link_h_prepare(const RawLink<P16>& r, float row3_factor, LinkH& L) {
  const unsigned e[9] = {r.q0.x, r.q0.y, r.q0.z, r.q0.w, r.q1.x, r.q1.y, r.q1.z, r.q1.w, r.t};
#pragma unroll
  for (int i = 0; i < 3 * ROWS; ++i) {
    L.p[i] = neg_hi(e[i]);
    L.s[i] = swap_halves(e[i]);
  }
  if constexpr (ROWS == 2) {
    // third row of s U (U in SU(3)) from the first two, in code units (the factor carries 1/s and the
    // link scale, as in rebuild_row3)
    Cx<float> u[9];
#pragma unroll
    for (int i = 0; i < 6; ++i) u[i] = unpack_h2(e[i], 1.f);
    rebuild_row3(u, row3_factor);
#pragma unroll
    for (int i = 0; i < 3; ++i) L.w[i] = u[6 + i];
  }
}

// acc += s (U v) for a link in dot2 form and the codes v0, v1, v2 of a colour vector; s = link scale x
// vector scale.  Per row: three chained dot2 for the real and three for the imaginary part (binary32
// code units), then one FMA each into the accumulator.
template <int ROWS>
__device__ __forceinline__ void matvec_h_acc(const LinkH& L, unsigned v0, unsigned v1, unsigned v2, float s,
                                             Cx<float> acc[3]) {
#pragma unroll
  for (int a = 0; a < ROWS; ++a) {
    float re = fdot2(L.p[3 * a], v0, 0.f);
    re = fdot2(L.p[3 * a + 1], v1, re);
    re = fdot2(L.p[3 * a + 2], v2, re);
    float im = fdot2(L.s[3 * a], v0, 0.f);
    im = fdot2(L.s[3 * a + 1], v1, im);
    im = fdot2(L.s[3 * a + 2], v2, im);
    acc[a].re = fmaf(s, re, acc[a].re);
    acc[a].im = fmaf(s, im, acc[a].im);
  }
  if constexpr (ROWS == 2) {
    const Cx<float> c[3] = {unpack_h2(v0, 1.f), unpack_h2(v1, 1.f), unpack_h2(v2, 1.f)};
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      re = fmaf(L.w[b].re, c[b].re, re);
      re = fmaf(-L.w[b].im, c[b].im, re);
      im = fmaf(L.w[b].re, c[b].im, im);
      im = fmaf(L.w[b].im, c[b].re, im);
    }
    acc[2].re = fmaf(s, re, acc[2].re);
    acc[2].im = fmaf(s, im, acc[2].im);
  }
}

// Order in which the FP16 Dslash accumulates the 16 matrices of an output site: the time hops
// -3, -1 first, then the x, y, z matrices, then the time hops +1, +3.  It is the order in which the
// time-streaming kernel (dslash_t.hip) receives them, so every FP16 launch shape gives the same bits.
__host__ __device__ constexpr int f16_link_order(int i) {
  return i == 0 ? 15 : (i == 1 ? 13 : (i < 14 ? i - 2 : (i == 14 ? 12 : 14)));
}

// Load the packed matrix k of the output site in block blk (lane = site % 64); C12: the three-hop
// matrices are stored as two rows (the caller rebuilds the third).  The layout is a compile-time
// choice so that the unrolled link loop stays straight-line code.
template <int P, bool C12>
__device__ __forceinline__ void load_link(const char* base, long blk, int k, int lane, float scale,
                                          Cx<typename RealOf<P>::T> u[9]) {
  const char* slot = base + link_slot_offset(P, C12, blk, k);
  if (C12 && (k & 3) >= 2)
    load_link_rows<P, 2>(slot, lane, scale, u);
  else
    load_link_rows<P, 3>(slot, lane, scale, u);
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
  if (mu == 3) cn = g.t_open ? (fwd ? c + h : c - h) : cn;  // a slab reads its ghost slices (a select)
  return s.cb + (cn - c) * g.stride[mu];
}

// Sign of eta_mu(n) s(start, 3) (times -1 for the backward term): the folded scalar of the three-hop
// matrix k = 4 mu + j (j = 2 forward, 3 backward) of output site s is c_N times this sign.
__device__ __forceinline__ int long_sign(const Site& s, const Geo& g, int mu, bool fwd) {
  const int eta_bits = mu == 0 ? 0 : (mu == 1 ? s.x : (mu == 2 ? s.x + s.y : s.x + s.y + s.z));
  int neg = (eta_bits & 1) ^ (fwd ? 0 : 1);
  if (mu == 3) {
    // floor((start + 3) / L_t) for 0 <= start < L_t, L_t >= 2, is (start+3 >= L_t) + (start+3 >= 2 L_t):
    // compares instead of a division or a branch keep the unrolled link loop straight-line code.
    // The time coordinate and extent are the whole lattice's (a slab adds its offset t0).
    const int tg = s.t + g.t0, Lg = g.lt_glob;
    const int start = fwd ? tg : wrap_bwd(tg, g.h3g, Lg);
    const int wraps = (start + 3 >= Lg) ^ (start + 3 >= 2 * Lg);
    neg ^= wraps & g.antiper;
  }
  return neg ? -1 : 1;
}

// ---- reductions ---------------------------------------------------------------
// Sum over the 64 lanes of a wave (butterfly of shuffles; every lane ends with the same sum).
template <int N> __device__ __forceinline__ void wave_sum(double v[N]) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, kWave);
}

// Deterministic block sum of N doubles per thread; the result is valid in thread 0.
template <int N, int MAXW = 4>
__device__ __forceinline__ void block_sum(double v[N], double* lds /* >= N * MAXW */) {
  wave_sum<N>(v);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (nw == 1) return;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) lds[i * MAXW + wave] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double s = lds[i * MAXW];
      for (int w = 1; w < nw; ++w) s += lds[i * MAXW + w];
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
