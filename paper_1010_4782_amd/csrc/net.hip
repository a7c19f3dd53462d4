// Kernels of the gauge-covariant linear network used as the flexible-CG preconditioner.
//
// A layer maps C_in colour-vector channels to C_out on the full lattice:
//   y_c(n) = sum_c' [ W_0[c][c'] psi_c'(n) + sum_{d=1..8} W_d[c][c'] (T_d psi_c')(n) ]
// with T_{+mu} psi(n) = F~_mu(n) psi(n+mu) and T_{-mu} psi(n) = F~_mu(n-mu)^dag psi(n-mu)
// (d = 1..4: +x,+y,+z,+t; d = 5..8: -x,-y,-z,-t).  The transports reuse the packed FP32
// one-hop matrices of the Dslash: for output parity p, k = 4 mu is F~_mu(n) and
// k = 4 mu + 1 is -F~_mu(n-mu)^dag, so T_{-mu} = -L_{4mu+1}.
//
// Activations are complex64, stored per parity.  With C >= 2 channels they are interleaved in
// channel pairs, [parity][C/2][V/2][3 colours][2 channels] (48 B per pair and site, three 16-byte
// loads), so that reading all channels of a neighbour takes 3C/2 wide loads instead of 3C narrow
// ones; a single channel is [parity][V/2][3].  A null input pointer stands for a field that is
// zero on that parity.
#include "device.h"
#include "net.h"
#include "launch.h"

namespace stag {

__device__ __forceinline__ void cmac_f(Cx<float>& acc, const float2 w, const Cx<float>& v) {
  acc.re = fmaf(w.x, v.re, acc.re);
  acc.re = fmaf(-w.y, v.im, acc.re);
  acc.im = fmaf(w.x, v.im, acc.im);
  acc.im = fmaf(w.y, v.re, acc.im);
}

// Channels c0 .. c0 + G - 1 of a C-channel activation at site cb (c0 even when G >= 2).
template <int C, int G>
__device__ __forceinline__ void load_channels(const float2* base, long half, long cb, int c0, Cx<float> t[G][3]) {
  if constexpr (C == 1) {
    load_spinor<P32>(base, cb, t[0]);
  } else {
    static_assert(G % 2 == 0, "channel pairs are loaded whole");
#pragma unroll
    for (int q = 0; q < G / 2; ++q) {
      gptr<f4v> p = as_global<f4v>(base + ((long)(c0 / 2 + q) * half + cb) * 6);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const f4v w = p[i];
        t[2 * q][i] = Cx<float>{w.x, w.y};
        t[2 * q + 1][i] = Cx<float>{w.z, w.w};
      }
    }
  }
}

template <int C>
__device__ __forceinline__ void store_channels(float2* base, long half, long cb, const Cx<float> v[C][3]) {
  if constexpr (C == 1) {
    gptr_w<f2v> p = as_global_w<f2v>(base + cb * 3);
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = f2v{v[0][i].re, v[0][i].im};
  } else {
#pragma unroll
    for (int q = 0; q < C / 2; ++q) {
      gptr_w<f4v> p = as_global_w<f4v>(base + ((long)q * half + cb) * 6);
#pragma unroll
      for (int i = 0; i < 3; ++i) p[i] = f4v{v[2 * q][i].re, v[2 * q][i].im, v[2 * q + 1][i].re, v[2 * q + 1][i].im};
    }
  }
}

// Transported colour vectors of all input channels along direction d (1..8) for the site s.
template <int CIN>
__device__ __forceinline__ void transported(const NetLayerArgs& a, const Site& s, long blk, int lane, int d,
                                            Cx<float> t[CIN][3]) {
  const int mu = (d - 1) & 3;
  const bool fwd = d <= 4;
  const int nb = neighbour(s, a.g, mu, a.g.h1[mu], fwd);
  Cx<float> u[9];
  if (a.g.long12)
    load_link<P32, true>(a.links, blk, 4 * mu + (fwd ? 0 : 1), lane, 1.f, u);
  else
    load_link<P32, false>(a.links, blk, 4 * mu + (fwd ? 0 : 1), lane, 1.f, u);
  if (!fwd)
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = Cx<float>{-u[e].re, -u[e].im};
  Cx<float> v[CIN][3];
  load_channels<CIN, CIN>(a.in_other, a.g.half, nb, 0, v);
#pragma unroll
  for (int c = 0; c < CIN; ++c) {
#pragma unroll
    for (int i = 0; i < 3; ++i) t[c][i] = Cx<float>{0.f, 0.f};
    matvec_acc(u, v[c], t[c]);
  }
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_layer(NetLayerArgs a) {
  const int cb_raw = blockIdx.x * blockDim.x + threadIdx.x;
  if (cb_raw >= a.g.half) return;
  const int cb = cb_raw;
  const Site s = site_of(cb, a.out_par, a.g);
  const long blk = cb >> 6;
  const int lane = cb & 63;
  Cx<float> acc[COUT][3];
#pragma unroll
  for (int c = 0; c < COUT; ++c)
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[c][i] = Cx<float>{0.f, 0.f};
  if (a.in_same) {
    Cx<float> v[CIN][3];
    load_channels<CIN, CIN>(a.in_same, a.g.half, cb, 0, v);
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) {
#pragma unroll
      for (int c = 0; c < COUT; ++c) {
        const float2 w = a.w[c * CIN + ci];
#pragma unroll
        for (int i = 0; i < 3; ++i) cmac_f(acc[c][i], w, v[ci][i]);
      }
    }
  }
  if (a.in_other) {
#pragma unroll 1
    for (int d = 1; d <= 8; ++d) {
      Cx<float> t[CIN][3];
      transported<CIN>(a, s, blk, lane, d, t);
      const float2* wd = a.w + d * COUT * CIN;
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
        for (int c = 0; c < COUT; ++c) {
          const float2 w = wd[c * CIN + ci];
#pragma unroll
          for (int i = 0; i < 3; ++i) cmac_f(acc[c][i], w, t[ci][i]);
        }
    }
  }
  store_channels<COUT>(a.out, a.g.half, cb, acc);
}

// Channel mixing on the matrix cores.  For the 64 sites of one wave and one term d (identity or a
// transport), the mixing is the complex product Y[c][n] += sum_c' W_d[c][c'] X_d[c'][n] over the
// 192 columns n = 3 site + colour.  It runs as a real GEMM with the 2x2 real form of each complex
// weight: rows i = 2c + {re, im}, inner index k = 2c' + {re, im},
//   A[2c][2c'] = Re W, A[2c][2c'+1] = -Im W, A[2c+1][2c'] = Im W, A[2c+1][2c'+1] = Re W,
// on v_mfma_f32_16x16x4_f32 (A 16x4, B 4x16, C 16x16 in FP32): twelve 16-column tiles, and
// ceil(CIN/2) steps of 4 inner indices per term.  The transports stay on the vector units, one
// lane per site, and reach the MFMA operand layout through LDS (12 KB per wave for CIN = 8).
//   MFMA lane layout (16x16x4): lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and
//   C[4 (l / 16) + r][l % 16], r = 0..3.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_layer_mfma(NetLayerArgs a) {
  static_assert(CIN >= 2 && CIN <= 8 && COUT >= 2 && COUT <= 8, "the matrix-core layer needs 2..8 channels");
  constexpr int KS = (CIN + 1) / 2;  // inner steps of 4 reals (2 input channels) per term
  constexpr int NT = 3 * kWave / 16;  // 16-column tiles per wave
  __shared__ float2 xs[256 / kWave][CIN][3 * kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int cb_raw = blockIdx.x * blockDim.x + threadIdx.x;
  const int wave_base = cb_raw - lane;
  if (wave_base >= a.g.half) return;  // whole wave past the lattice (uniform per wave)
  const bool live = cb_raw < a.g.half;
  const int cb = live ? cb_raw : a.g.half - 1;  // dead lanes compute a valid site; their columns are not stored
  const Site s = site_of(cb, a.out_par, a.g);
  const int row = lane & 15, kq = lane >> 4;
  f4v acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
  float* xw = reinterpret_cast<float*>(&xs[wave][0][0]);
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    if (d == 0 ? a.in_same == nullptr : a.in_other == nullptr) continue;  // uniform
    Cx<float> t[CIN][3];
    if (d == 0) {
      load_channels<CIN, CIN>(a.in_same, a.g.half, cb, 0, t);
    } else {
      transported<CIN>(a, s, cb >> 6, cb & 63, d, t);
    }
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
      for (int i = 0; i < 3; ++i) xs[wave][ci][3 * lane + i] = make_float2(t[ci][i].re, t[ci][i].im);
    __builtin_amdgcn_wave_barrier();
    // A operand of this lane: row `row`, inner index 4 ks + kq
    float av[KS];
    {
      const int c = row >> 1, ri = row & 1;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + kq, cp = k >> 1, ki = k & 1;
        float v = 0.f;
        if (c < COUT && cp < CIN) {
          const float2 w = a.w[(d * COUT + c) * CIN + cp];
          v = ri == 0 ? (ki == 0 ? w.x : -w.y) : (ki == 0 ? w.y : w.x);
        }
        av[ks] = v;
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cp = 2 * ks + (kq >> 1), ki = kq & 1;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const float bv = cp < CIN ? xw[(cp * 3 * kWave + 16 * j + row) * 2 + ki] : 0.f;
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], bv, acc[j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // C rows 4 kq .. 4 kq + 3 are channels 2 kq and 2 kq + 1, (re, im) each; column 16 j + row.
  static_assert(COUT % 2 == 0, "matrix-core layers write whole channel pairs");
  const int c0 = 2 * kq;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int n = 16 * j + row;
    const int site = wave_base + n / 3, colour = n % 3;
    if (site >= a.g.half || c0 >= COUT) continue;
    // channels c0, c0 + 1 are one pair of the interleaved layout: one 16-byte store
    as_global_w<f4v>(a.out + ((long)kq * a.g.half + site) * 6)[colour] = acc[j];
  }
}

// Weight gradient, one direction d (blockIdx.y) and a group of G output channels (blockIdx.z):
//   partial[p][d][c][c'] = sum_n sum_a G_c(n)_a conj((T_d psi_c')(n)_a)
// over the output sites of parity a.out_par; each block walks sites with a grid stride and
// writes one partial (complex, FP64) per (d, c, c') for a fixed-order second stage.
template <int CIN, int COUT, int G>
__global__ __launch_bounds__(256) void k_net_wgrad(NetLayerArgs a, const float2* gy, double* partial) {
  const int d = blockIdx.y;
  const int cg = blockIdx.z;
  Cx<float> acc[G][CIN];
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) acc[c][ci] = Cx<float>{0.f, 0.f};
  const bool have = d == 0 ? a.in_same != nullptr : a.in_other != nullptr;
  if (have && gy) {
    for (int cb = blockIdx.x * blockDim.x + threadIdx.x; cb < a.g.half; cb += gridDim.x * blockDim.x) {
      const Site s = site_of(cb, a.out_par, a.g);
      Cx<float> t[CIN][3];
      if (d == 0) {
        load_channels<CIN, CIN>(a.in_same, a.g.half, cb, 0, t);
      } else {
        transported<CIN>(a, s, cb >> 6, cb & 63, d, t);
      }
      Cx<float> gvs[G][3];
      load_channels<COUT, G>(gy, a.g.half, cb, cg * G, gvs);
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const Cx<float>* gv = gvs[c];
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            // g * conj(t)
            acc[c][ci].re = fmaf(gv[i].re, t[ci][i].re, acc[c][ci].re);
            acc[c][ci].re = fmaf(gv[i].im, t[ci][i].im, acc[c][ci].re);
            acc[c][ci].im = fmaf(gv[i].im, t[ci][i].re, acc[c][ci].im);
            acc[c][ci].im = fmaf(-gv[i].re, t[ci][i].im, acc[c][ci].im);
          }
      }
    }
  }
  // block reduction, one (c, c') pair at a time, in FP64
  __shared__ double lds[2 * 4];
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) {
      double v[2] = {(double)acc[c][ci].re, (double)acc[c][ci].im};
      block_sum<2>(v, lds);
      if (threadIdx.x == 0) {
        const int co = cg * G + c;
        const long idx = ((((long)a.out_par * 9 + d) * COUT + co) * CIN + ci) * gridDim.x + blockIdx.x;
        partial[2 * idx] = v[0];
        partial[2 * idx + 1] = v[1];
      }
      __syncthreads();
    }
}

// Weight gradient on the matrix cores, one direction d per blockIdx.y:
//   P[c][c'] = sum_n sum_a G_c(n)_a conj(X_d,c'(n)_a),  X_d = T_d psi (or psi for d = 0),
// as a real GEMM over the inner index k = 2 n + part (n = 3 site + colour) with rows i = 2c + {re, im}:
//   A[2c][(n,0)] = Re G, A[2c][(n,1)] = Im G, A[2c+1][(n,0)] = Im G, A[2c+1][(n,1)] = -Re G,
//   B[(n,0)][c'] = Re X, B[(n,1)][c'] = Im X   (columns c' >= CIN are zero).
// Each wave walks 64-site chunks with a grid stride and accumulates one 16x16 FP32 tile; the waves
// of a block are summed in FP64 in a fixed order and written as one partial per block in the
// layout of k_net_wgrad.
constexpr int kWgradMfmaWG = 128;  // two waves: 52 KB of LDS per workgroup at 8 channels, three per CU

template <int CIN, int COUT>
__global__ __launch_bounds__(kWgradMfmaWG) void k_net_wgrad_mfma(NetLayerArgs a, const float2* gy, double* partial) {
  static_assert(CIN >= 2 && CIN <= 8 && COUT >= 2 && COUT <= 8, "the matrix-core gradient needs 2..8 channels");
  constexpr int NW = kWgradMfmaWG / kWave;
  __shared__ float2 xs[NW][CIN][3 * kWave];
  __shared__ float2 gs[NW][COUT][3 * kWave];
  __shared__ double red[NW][kWave][4];
  const int d = blockIdx.y;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int row = lane & 15, kq = lane >> 4;
  f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
  const bool have = d == 0 ? a.in_same != nullptr : a.in_other != nullptr;
  const float* xw = reinterpret_cast<const float*>(&xs[wave][0][0]);
  const float* gw = reinterpret_cast<const float*>(&gs[wave][0][0]);
  if (have && gy) {
    const int nchunk = ceil_div(a.g.half, kWave);
    for (int ch = blockIdx.x * NW + wave; ch < nchunk; ch += gridDim.x * NW) {  // uniform per wave
      const int cb_raw = ch * kWave + lane;
      const bool live = cb_raw < a.g.half;
      const int cb = live ? cb_raw : a.g.half - 1;
      Cx<float> t[CIN][3];
      if (d == 0) {
        load_channels<CIN, CIN>(a.in_same, a.g.half, cb, 0, t);
      } else {
        const Site s = site_of(cb, a.out_par, a.g);
        transported<CIN>(a, s, cb >> 6, cb & 63, d, t);
      }
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          xs[wave][ci][3 * lane + i] = live ? make_float2(t[ci][i].re, t[ci][i].im) : make_float2(0.f, 0.f);
      Cx<float> gvs[COUT][3];
      load_channels<COUT, COUT>(gy, a.g.half, cb, 0, gvs);
#pragma unroll
      for (int c = 0; c < COUT; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          gs[wave][c][3 * lane + i] = live ? make_float2(gvs[c][i].re, gvs[c][i].im) : make_float2(0.f, 0.f);
      __builtin_amdgcn_wave_barrier();
      // inner step ks covers n = 2 ks + (kq >> 1), part = kq & 1
      const int c = row >> 1, ri = row & 1, part = kq & 1;
#pragma unroll 8
      for (int ks = 0; ks < 3 * kWave / 2; ++ks) {
        const int n = 2 * ks + (kq >> 1);
        float av = 0.f, bv = 0.f;
        if (c < COUT) {
          const float gr = gw[(c * 3 * kWave + n) * 2], gi = gw[(c * 3 * kWave + n) * 2 + 1];
          av = ri == 0 ? (part == 0 ? gr : gi) : (part == 0 ? gi : -gr);
        }
        if (row < CIN) bv = xw[(row * 3 * kWave + n) * 2 + part];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave][lane][r] = (double)acc[r];
  __syncthreads();
  if (wave != 0) return;
  double v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    v[r] = red[0][lane][r];
    for (int w = 1; w < NW; ++w) v[r] += red[w][lane][r];
  }
  // C rows 4 kq + r: channel 2 kq + (r >> 1), part r & 1; column row = c'
  const int cp = row;
  if (cp >= CIN) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int co = 2 * kq + h;
    if (co >= COUT) continue;
    const long idx = ((((long)a.out_par * 9 + d) * COUT + co) * CIN + cp) * gridDim.x + blockIdx.x;
    partial[2 * idx] = v[2 * h];
    partial[2 * idx + 1] = v[2 * h + 1];
  }
}

// out[d][c][c'] = sum over parities and blocks of the partials, in a fixed order.
__global__ __launch_bounds__(64) void k_net_wgrad_reduce(const double* partial, int cin, int cout, int nblk,
                                                         int npar, double* out) {  // out += sum
  const int j = blockIdx.x * blockDim.x + threadIdx.x;  // (d, c, c') flat
  const int n = 9 * cout * cin;
  if (j >= n) return;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < npar; ++p)
    for (int b = 0; b < nblk; ++b) {
      const long idx = ((long)p * n + j) * nblk + b;
      re += partial[2 * idx];
      im += partial[2 * idx + 1];
    }
  out[2 * j] += re;
  out[2 * j + 1] += im;
}

// even-site complex128 vector -> channel 0 of a complex64 activation (parity 0)
__global__ __launch_bounds__(256) void k_net_embed(const double2* in, float2* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = in[i];
  out[i] = make_float2((float)v.x, (float)v.y);
}

// channel 0 of a complex64 activation (parity 0) -> even-site complex128 vector
__global__ __launch_bounds__(256) void k_net_extract(const float2* in, double2* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 v = in[i];
  out[i] = make_double2((double)v.x, (double)v.y);
}

// Loss gradient at the output: g = scale (N(b) - x) on even sites; partial |N(b) - x|^2 per block.
__global__ __launch_bounds__(256) void k_net_loss(const float2* out, const double2* x, double scale, float2* g,
                                                  double* partial, long n) {
  __shared__ double lds[4];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double s[1] = {0.0};
  if (i < n) {
    const float2 o = out[i];
    const double2 xv = x[i];
    const double dr = (double)o.x - xv.x, di = (double)o.y - xv.y;
    s[0] = dr * dr + di * di;
    g[i] = make_float2((float)(scale * dr), (float)(scale * di));
  }
  block_sum<1>(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double lds[4];
  double s[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) s[0] += partial[i];
  block_sum<1>(s, lds);
  if (threadIdx.x == 0) *out = s[0];
}

// ---- launchers ---------------------------------------------------------------------
hipError_t launch_net_layer(const NetLayerArgs& a, int cin, int cout, hipStream_t st) {
  const int nb = ceil_div(a.g.half, 256);
  // layers with at least two channels on both sides mix on the matrix cores; 1 -> C and C -> 1
  // would fill at most a quarter of an MFMA tile and stay on the vector units
#define STAG_NET_LAYER(I, O) \
  if (cin == I && cout == O) { k_net_layer<I, O><<<nb, 256, 0, st>>>(a); return hipGetLastError(); }
#define STAG_NET_LAYER_MFMA(I, O) \
  if (cin == I && cout == O) { k_net_layer_mfma<I, O><<<nb, 256, 0, st>>>(a); return hipGetLastError(); }
  STAG_NET_LAYER(1, 1) STAG_NET_LAYER(1, 2) STAG_NET_LAYER(2, 1) STAG_NET_LAYER_MFMA(2, 2)
  STAG_NET_LAYER(1, 4) STAG_NET_LAYER(4, 1) STAG_NET_LAYER_MFMA(4, 4)
  STAG_NET_LAYER(1, 8) STAG_NET_LAYER(8, 1) STAG_NET_LAYER_MFMA(8, 8)
#undef STAG_NET_LAYER
#undef STAG_NET_LAYER_MFMA
  return hipErrorInvalidValue;
}

hipError_t launch_net_wgrad(const NetLayerArgs& a, const float2* gy, double* partial, int cin, int cout, int nblk,
                            hipStream_t st) {
#define STAG_NET_WG(I, O, G)                                                  \
  if (cin == I && cout == O) {                                                \
    k_net_wgrad<I, O, G><<<dim3(nblk, 9, O / G), 256, 0, st>>>(a, gy, partial); \
    return hipGetLastError();                                                 \
  }
#define STAG_NET_WG_MFMA(I, O)                                                       \
  if (cin == I && cout == O) {                                                       \
    k_net_wgrad_mfma<I, O><<<dim3(nblk, 9, 1), kWgradMfmaWG, 0, st>>>(a, gy, partial); \
    return hipGetLastError();                                                        \
  }
  STAG_NET_WG(1, 1, 1) STAG_NET_WG(1, 2, 2) STAG_NET_WG(2, 1, 1) STAG_NET_WG_MFMA(2, 2)
  STAG_NET_WG(1, 4, 4) STAG_NET_WG(4, 1, 1) STAG_NET_WG_MFMA(4, 4)
  STAG_NET_WG(1, 8, 8) STAG_NET_WG(8, 1, 1) STAG_NET_WG_MFMA(8, 8)
#undef STAG_NET_WG
#undef STAG_NET_WG_MFMA
  return hipErrorInvalidValue;
}

hipError_t launch_net_wgrad_reduce(const double* partial, int cin, int cout, int nblk, int npar, double* out,
                                   hipStream_t st) {
  const int n = 9 * cout * cin;
  k_net_wgrad_reduce<<<ceil_div(n, 64), 64, 0, st>>>(partial, cin, cout, nblk, npar, out);
  return hipGetLastError();
}

hipError_t launch_net_embed(const void* in, float2* out, long nsites, hipStream_t st) {
  const long n = nsites * 3;
  if (n == 0) return hipSuccess;
  k_net_embed<<<(n + 255) / 256, 256, 0, st>>>(reinterpret_cast<const double2*>(in), out, n);
  return hipGetLastError();
}

hipError_t launch_net_extract(const float2* in, void* out, long nsites, hipStream_t st) {
  const long n = nsites * 3;
  if (n == 0) return hipSuccess;
  k_net_extract<<<(n + 255) / 256, 256, 0, st>>>(in, reinterpret_cast<double2*>(out), n);
  return hipGetLastError();
}

hipError_t launch_net_loss(const float2* out, const void* x, double scale, float2* g, double* partial, double* sum,
                           long nsites, hipStream_t st) {
  const long n = nsites * 3;
  const int nb = (int)((n + 255) / 256);
  k_net_loss<<<nb, 256, 0, st>>>(out, reinterpret_cast<const double2*>(x), scale, g, partial, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials<<<1, 256, 0, st>>>(partial, nb, sum);
  return hipGetLastError();
}

}  // namespace stag

namespace stag {

__global__ __launch_bounds__(256) void k_norm2_c128(const double2* x, double* partial, long n) {
  __shared__ double lds[4];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double s[1] = {0.0};
  if (i < n) {
    const double2 v = x[i];
    s[0] = v.x * v.x + v.y * v.y;
  }
  block_sum<1>(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

hipError_t launch_norm2_c128(const void* x, double* partial, double* sum, long nsites, hipStream_t st) {
  const long n = nsites * 3;
  const int nb = (int)((n + 255) / 256);
  k_norm2_c128<<<nb, 256, 0, st>>>(reinterpret_cast<const double2*>(x), partial, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials<<<1, 256, 0, st>>>(partial, nb, sum);
  return hipGetLastError();
}

}  // namespace stag

namespace stag {

// out = a - b (complex128), partial |out|^2 per block
__global__ __launch_bounds__(256) void k_sub_norm(const double2* a, const double2* b, double2* out, double* partial,
                                                  long n) {
  __shared__ double lds[4];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double s[1] = {0.0};
  if (i < n) {
    const double2 u = a[i], v = b[i];
    const double2 w = make_double2(u.x - v.x, u.y - v.y);
    out[i] = w;
    s[0] = w.x * w.x + w.y * w.y;
  }
  block_sum<1>(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// complex128 -> complex64 times a real scale
__global__ __launch_bounds__(256) void k_scale_to_f32(const double2* in, double scale, float2* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = in[i];
  out[i] = make_float2((float)(scale * v.x), (float)(scale * v.y));
}

hipError_t launch_sub_norm(const void* a, const void* b, void* out, double* partial, double* sum, long nsites,
                           hipStream_t st) {
  const long n = nsites * 3;
  const int nb = (int)((n + 255) / 256);
  k_sub_norm<<<nb, 256, 0, st>>>(reinterpret_cast<const double2*>(a), reinterpret_cast<const double2*>(b),
                                 reinterpret_cast<double2*>(out), partial, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_partials<<<1, 256, 0, st>>>(partial, nb, sum);
  return hipGetLastError();
}

hipError_t launch_scale_to_f32(const void* in, double scale, float2* out, long nsites, hipStream_t st) {
  const long n = nsites * 3;
  k_scale_to_f32<<<(n + 255) / 256, 256, 0, st>>>(reinterpret_cast<const double2*>(in), scale, out, n);
  return hipGetLastError();
}

}  // namespace stag
