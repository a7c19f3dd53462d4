// Fused CG vector stages and deterministic reductions (Fig. 1's vector algebra).
//
// Each stage is one launch over every right-hand side ("slot") of the batch.
// Reductions are two-stage and deterministic: a wave64 shuffle tree plus an
// LDS step per workgroup write one partial per (slot, tile); a finalize launch
// with one workgroup per slot sums the partials in a fixed order and updates
// the slot's FP64 scalars (alpha, beta, stopping state) on the device, so the
// host never waits inside an iteration.
#include "device.h"
#include "launch.h"

namespace stag {

struct VecMap {
  const ProbDev* pd;
  int p, tile, r, slot, cb;
  bool live;
};

__device__ __forceinline__ bool map_vec_block(const Batch& B, VecMap& m) {
  const int bid = blockIdx.x;
  m.p = find_problem(B, bid);
  m.pd = B.probs + m.p;
  const int local = bid - B.block_start[m.p];
  const int groups = B.groups[m.p];
  m.tile = local / groups;
  m.r = local - m.tile * groups;
  m.slot = m.pd->slot0 + m.r;
  const int cb = m.tile * blockDim.x + threadIdx.x;
  m.live = cb < m.pd->g.half;
  m.cb = m.live ? cb : 0;
  return true;
}

template <int P>
__device__ __forceinline__ char* vec_ptr(const VecMap& m, int id) {
  return reinterpret_cast<char*>(m.pd->vec[id]) + (long)m.r * m.pd->g.half * spinor_bytes(P);
}

__device__ __forceinline__ void write_partial(const Batch& B, const VecMap& m, int kind, double v) {
  if (threadIdx.x == 0) B.partial[((long)m.slot * kPartialSlots + kind) * B.pstride + m.tile] = v;
}

// partial[kind] = |v|^2
template <int P>
__global__ __launch_bounds__(kMaxWG) void k_norm2(Batch B, int v_id, int kind, int gate) {
  __shared__ double lds[4];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate)) return;
  double s[1] = {0.0};
  if (m.live) {
    Cx<typename RealOf<P>::T> v[3];
    load_spinor<P>(vec_ptr<P>(m, v_id), m.cb, v);
#pragma unroll
    for (int c = 0; c < 3; ++c) s[0] += (double)v[c].re * v[c].re + (double)v[c].im * v[c].im;
  }
  block_sum<1>(s, lds);
  write_partial(B, m, kind, s[0]);
}

// r -= alpha Ad ; partial[1] = |r|^2 (of the stored r)
template <int P>
__global__ __launch_bounds__(kMaxWG) void k_update_r(Batch B, int r_id, int ad_id) {
  using T = typename RealOf<P>::T;
  // Streamed once: non-temporal for the storage-precision vectors (0.8% off the 8-RHS mixed-precision
  // solve at 48^3x144); the FP64 CG keeps the default, with which its 8-RHS solve is 7% faster.
  constexpr bool kNT = P != P64;
  __shared__ double lds[4];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, 1)) return;
  const T alpha = (T)B.scal[m.slot].alpha;
  double s[1] = {0.0};
  if (m.live) {
    Cx<T> r[3], a[3];
    char* rp = vec_ptr<P>(m, r_id);
    load_spinor<P, kNT>(rp, m.cb, r);
    load_spinor<P, kNT>(vec_ptr<P>(m, ad_id), m.cb, a);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c].re = fma(-alpha, a[c].re, r[c].re);
      r[c].im = fma(-alpha, a[c].im, r[c].im);
    }
    store_spinor<P, kNT>(rp, m.cb, r);
#pragma unroll
    for (int c = 0; c < 3; ++c) s[0] += (double)r[c].re * r[c].re + (double)r[c].im * r[c].im;
  }
  block_sum<1>(s, lds);
  write_partial(B, m, 1, s[0]);
}

// x += alpha d (x in precision PX) ; d = r + beta d
template <int P, int PX>
__global__ __launch_bounds__(kMaxWG) void k_update_xd(Batch B, int x_id, int r_id, int d_id) {
  using T = typename RealOf<P>::T;
  using TX = typename RealOf<PX>::T;
  constexpr bool kNT = P != P64;  // as in k_update_r
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, 2) || !m.live) return;
  const Scal& sc = B.scal[m.slot];
  const TX alpha = (TX)sc.alpha;
  const T beta = (T)sc.beta;
  Cx<T> d[3], r[3];
  Cx<TX> x[3];
  char* dp = vec_ptr<P>(m, d_id);
  char* xp = vec_ptr<PX>(m, x_id);
  load_spinor<P, kNT>(dp, m.cb, d);
  load_spinor<P, kNT>(vec_ptr<P>(m, r_id), m.cb, r);
  load_spinor<PX, kNT>(xp, m.cb, x);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[c].re = fma(alpha, (TX)d[c].re, x[c].re);
    x[c].im = fma(alpha, (TX)d[c].im, x[c].im);
    d[c].re = fma(beta, d[c].re, r[c].re);
    d[c].im = fma(beta, d[c].im, r[c].im);
  }
  store_spinor<PX, kNT>(xp, m.cb, x);
  store_spinor<P, kNT>(dp, m.cb, d);
}

template <int PS, int PD>
__global__ __launch_bounds__(kMaxWG) void k_copy(Batch B, int src_id, int dst_id, int gate) {
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate) || !m.live) return;
  Cx<typename RealOf<PS>::T> a[3];
  load_spinor<PS>(vec_ptr<PS>(m, src_id), m.cb, a);
  Cx<typename RealOf<PD>::T> b[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) b[c] = {(typename RealOf<PD>::T)a[c].re, (typename RealOf<PD>::T)a[c].im};
  store_spinor<PD>(vec_ptr<PD>(m, dst_id), m.cb, b);
}

// x (f64) += x_lo (f32) ; x_lo = 0
__global__ __launch_bounds__(kMaxWG) void k_add_lo_to_hi(Batch B, int gate) {
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate) || !m.live) return;
  Cx<double> x[3];
  Cx<float> xl[3];
  char* xp = vec_ptr<P64>(m, V_X);
  char* lp = vec_ptr<P32>(m, V_XL);
  load_spinor<P64>(xp, m.cb, x);
  load_spinor<P32>(lp, m.cb, xl);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[c].re += (double)xl[c].re;
    x[c].im += (double)xl[c].im;
    xl[c] = {0.f, 0.f};
  }
  store_spinor<P64>(xp, m.cb, x);
  store_spinor<P32>(lp, m.cb, xl);
}

template <int P>
__global__ __launch_bounds__(kMaxWG) void k_zero(Batch B, int v_id, int gate) {
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate) || !m.live) return;
  Cx<typename RealOf<P>::T> z[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) z[c] = {0, 0};
  store_spinor<P>(vec_ptr<P>(m, v_id), m.cb, z);
}

// partial[0,1,2] = Re <r, d>, Im <r, d>, |r|^2 with r the low-precision residual.
template <int P>
__global__ __launch_bounds__(kMaxWG) void k_rd_dot(Batch B, int gate) {
  __shared__ double lds[12];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate)) return;
  double s[3] = {0.0, 0.0, 0.0};
  if (m.live) {
    Cx<typename RealOf<P>::T> r[3], d[3];
    load_spinor<P>(vec_ptr<P>(m, V_RL), m.cb, r);
    load_spinor<P>(vec_ptr<P>(m, V_D), m.cb, d);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s[0] += (double)r[c].re * d[c].re + (double)r[c].im * d[c].im;
      s[1] += (double)r[c].re * d[c].im - (double)r[c].im * d[c].re;
      s[2] += (double)r[c].re * r[c].re + (double)r[c].im * r[c].im;
    }
  }
  block_sum<3>(s, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) B.partial[((long)m.slot * kPartialSlots + k) * B.pstride + m.tile] = s[k];
}

// d += c r with c = 1 - <r, d>/|r|^2 (from FIN_ORTHO): afterwards <r, d> = |r|^2 as in exact CG.
template <int P>
__global__ __launch_bounds__(kMaxWG) void k_d_fix(Batch B, int gate) {
  using T = typename RealOf<P>::T;
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate) || !m.live) return;
  const T cr = (T)B.scal[m.slot].cre, ci = (T)B.scal[m.slot].cim;
  Cx<T> r[3], d[3];
  char* dp = vec_ptr<P>(m, V_D);
  load_spinor<P>(vec_ptr<P>(m, V_RL), m.cb, r);
  load_spinor<P>(dp, m.cb, d);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    d[c].re += cr * r[c].re - ci * r[c].im;
    d[c].im += cr * r[c].im + ci * r[c].re;
  }
  store_spinor<P>(dp, m.cb, d);
}

// ---- flexible CG (FP64 vectors) ----------------------------------------------------
// d = z + beta d (complex beta from FIN_FCG_BETA; 0 on the first iteration); partial kinds 1, 2 = Re, Im <d, r>.
__global__ __launch_bounds__(kMaxWG) void k_fcg_dir(Batch B, int gate) {
  __shared__ double lds[8];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate)) return;
  const double br = B.scal[m.slot].br, bi = B.scal[m.slot].bi;
  double s[2] = {0.0, 0.0};
  if (m.live) {
    Cx<double> z[3], d[3], r[3];
    char* dp = vec_ptr<P64>(m, V_D);
    load_spinor<P64>(dp, m.cb, d);
    load_spinor<P64>(vec_ptr<P64>(m, V_R), m.cb, r);
    load_spinor<P64>(vec_ptr<P64>(m, V_Z), m.cb, z);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      d[c] = Cx<double>{z[c].re + br * d[c].re - bi * d[c].im, z[c].im + br * d[c].im + bi * d[c].re};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s[0] += d[c].re * r[c].re + d[c].im * r[c].im;
      s[1] += d[c].re * r[c].im - d[c].im * r[c].re;
    }
    store_spinor<P64>(dp, m.cb, d);
  }
  block_sum<2>(s, lds);
  if (threadIdx.x == 0) {
    B.partial[((long)m.slot * kPartialSlots + 1) * B.pstride + m.tile] = s[0];
    B.partial[((long)m.slot * kPartialSlots + 2) * B.pstride + m.tile] = s[1];
  }
}

// x += alpha d ; r -= alpha Ad (complex alpha) ; partial kind 1 = |r|^2
__global__ __launch_bounds__(kMaxWG) void k_fcg_update(Batch B) {
  __shared__ double lds[4];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, 1)) return;
  const double ar = B.scal[m.slot].ar, ai = B.scal[m.slot].ai;
  double s[1] = {0.0};
  if (m.live) {
    Cx<double> x[3], d[3], r[3], a[3];
    char* xp = vec_ptr<P64>(m, V_X);
    char* rp = vec_ptr<P64>(m, V_R);
    load_spinor<P64>(xp, m.cb, x);
    load_spinor<P64>(vec_ptr<P64>(m, V_D), m.cb, d);
    load_spinor<P64>(rp, m.cb, r);
    load_spinor<P64>(vec_ptr<P64>(m, V_AD), m.cb, a);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c].re += ar * d[c].re - ai * d[c].im;
      x[c].im += ar * d[c].im + ai * d[c].re;
      r[c].re -= ar * a[c].re - ai * a[c].im;
      r[c].im -= ar * a[c].im + ai * a[c].re;
      s[0] += r[c].re * r[c].re + r[c].im * r[c].im;
    }
    store_spinor<P64>(xp, m.cb, x);
    store_spinor<P64>(rp, m.cb, r);
  }
  block_sum<1>(s, lds);
  write_partial(B, m, 1, s[0]);
}

// partial kinds 1, 2 = Re, Im <Ad, z>
__global__ __launch_bounds__(kMaxWG) void k_fcg_beta_dot(Batch B, int gate) {
  __shared__ double lds[8];
  VecMap m;
  map_vec_block(B, m);
  if (!slot_on(B.scal, m.slot, gate)) return;
  double s[2] = {0.0, 0.0};
  if (m.live) {
    Cx<double> a[3], z[3];
    load_spinor<P64>(vec_ptr<P64>(m, V_AD), m.cb, a);
    load_spinor<P64>(vec_ptr<P64>(m, V_Z), m.cb, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s[0] += a[c].re * z[c].re + a[c].im * z[c].im;
      s[1] += a[c].re * z[c].im - a[c].im * z[c].re;
    }
  }
  block_sum<2>(s, lds);
  if (threadIdx.x == 0) {
    B.partial[((long)m.slot * kPartialSlots + 1) * B.pstride + m.tile] = s[0];
    B.partial[((long)m.slot * kPartialSlots + 2) * B.pstride + m.tile] = s[1];
  }
}

// One workgroup per slot: sum the partials of `kind` in a fixed order and apply `what`.  The
// partials (about 2^14 per slot for a 28^3x96 Dslash of 64-site workgroups) come from HBM after the
// producing launch, so the kernel is a chain of memory round trips.  It is kept short: the problem
// size and the slot scalars that the per-iteration alpha and beta steps read are requested together
// at the start, and 16 waves issue all their loads (up to 24 per lane, one pass up to 24576
// partials) before the first add.  Lane t adds the partials t, t + 1024, t + 2048, ... in that order
// whatever the number of passes, so the sum does not depend on the unroll depth.
constexpr int kFinWG = 1024;
constexpr int kFinUnroll = 24;
__global__ __launch_bounds__(kFinWG) void k_finalize(Batch B, int what, int kind, int gate, int producer_wg,
                                                     int aux_wg, double* hist, int hist_stride) {
  __shared__ double lds[3 * (kFinWG / kWave)];
  const int slot = blockIdx.x;
  int p = 0;
  while (p + 1 < B.nprob && slot >= B.probs[p + 1].slot0) ++p;
  const Scal& pre = B.scal[slot];
  const int st = pre.state, iter0 = pre.iter, max_iter0 = pre.max_iter;
  const double delta0 = pre.delta, thr0 = pre.thr, rel_thr0 = pre.rel_thr;
  const int half = B.probs[p].g.half;
  if (!slot_on(B.scal, slot, gate)) return;
  const int nk = (what == FIN_ORTHO || what == FIN_FCG_ALPHA) ? 3 : (what == FIN_FCG_BETA ? 2 : 1);
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < nk; ++k) {
    // the first kind comes from a launch of producer_wg sites per block, the others from aux_wg
    const int ntiles = ceil_div(half, k == 0 ? producer_wg : aux_wg);
    const double* src = B.partial + ((long)slot * kPartialSlots + kind + k) * B.pstride;
    double v[kFinUnroll];
    for (int base = 0; base < ntiles; base += kFinUnroll * kFinWG) {
#pragma unroll
      for (int j = 0; j < kFinUnroll; ++j) {
        const int i = base + j * kFinWG + threadIdx.x;
        v[j] = i < ntiles ? src[i] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kFinUnroll; ++j) s[k] += v[j];
    }
  }
  block_sum<3, kFinWG / kWave>(s, lds);
  if (threadIdx.x != 0) return;
  const double sum = s[0];
  Scal& sc = B.scal[slot];
  switch (what) {
    case FIN_B2:
      sc.b2 = sum;
      sc.thr = sc.aux * sum;  // aux holds tol^2
      break;
    case FIN_START:
      sc.delta = sum;
      sc.iter = 0;
      sc.flags &= ~kFlagMaxIter;
      if (!isfinite(sum)) {
        sc.flags |= kFlagNaN;
        sc.state = 2;
      } else {
        sc.state = sum <= sc.thr ? 2 : 0;
      }
      break;
    case FIN_ALPHA: {
      if (st == 1) {
        sc.state = 2;
        break;
      }
      if (st != 0) break;
      sc.dAd = sum;
      if (!(sum > 0.0) || !isfinite(sum)) {
        sc.flags |= kFlagNaN;
        sc.state = 2;
        break;
      }
      const double alpha = delta0 / sum;
      sc.alpha = alpha;
      if (hist && iter0 < sc.hist_len) hist[((long)slot * hist_stride + iter0) * 2] = alpha;
      break;
    }
    case FIN_BETA: {
      if (st != 0) break;
      if (!isfinite(sum)) {
        sc.flags |= kFlagNaN;
        sc.state = 2;
        break;
      }
      const double beta = sum / delta0;
      sc.delta_old = delta0;
      sc.delta = sum;
      sc.beta = beta;
      if (hist && iter0 < sc.hist_len) hist[((long)slot * hist_stride + iter0) * 2 + 1] = beta;
      sc.iter = iter0 + 1;
      if (sum <= thr0) sc.state = 1;
      if (sum <= rel_thr0) {
        sc.state = 1;
        sc.flags |= kFlagRelDue;
      }
      if (iter0 + 1 >= max_iter0) {
        sc.state = 1;
        sc.flags |= kFlagMaxIter;
      }
      break;
    }
    case FIN_TRUE:
      sc.aux = sqrt(sum / sc.b2);
      sc.delta = sum;
      break;
    case FIN_RELIABLE:
      sc.delta = sum;
      break;
    case FIN_FCG_ALPHA:
      if (sc.state != 0) break;
      sc.dAd = sum;
      if (!(sum > 0.0) || !isfinite(sum) || !isfinite(s[1]) || !isfinite(s[2])) {
        sc.flags |= kFlagBreakdown;
        sc.state = 2;
        break;
      }
      sc.ar = s[1] / sum;
      sc.ai = s[2] / sum;
      if (hist && sc.iter < sc.hist_len) hist[((long)slot * hist_stride + sc.iter) * 2] = sc.ar;
      break;
    case FIN_FCG_RES:
      if (sc.state != 0) break;
      if (!isfinite(sum)) {
        sc.flags |= kFlagBreakdown;
        sc.state = 2;
        break;
      }
      sc.delta_old = sc.delta;
      sc.delta = sum;
      sc.dmin = fmin(sc.dmin, sum);
      sc.iter += 1;
      if (sum <= sc.thr) sc.state = 1;
      if (sc.iter >= sc.max_iter) {
        sc.state = 1;
        sc.flags |= kFlagMaxIter;
      }
      break;
    case FIN_FCG_BETA:
      if (sc.state != 0) break;
      sc.br = -sum / sc.dAd;
      sc.bi = -s[1] / sc.dAd;
      break;
    case FIN_ORTHO: {
      const double n2 = s[2];
      if (n2 > 0.0 && isfinite(n2)) {
        sc.cre = 1.0 - sum / n2;
        sc.cim = -s[1] / n2;
      } else {
        sc.cre = 0.0;
        sc.cim = 0.0;
      }
      sc.delta = n2;
      break;
    }
  }
}

// ---- launchers ------------------------------------------------------------------
static inline int nblocks(const Batch& B) { return B.block_start[B.nprob]; }

#define STAG_PREC_SWITCH(prec, KERNEL, ...)                     \
  switch (prec) {                                               \
    case P64: KERNEL<P64><<<nb, wg, 0, st>>>(__VA_ARGS__); break; \
    case P32: KERNEL<P32><<<nb, wg, 0, st>>>(__VA_ARGS__); break; \
    case P16: KERNEL<P16><<<nb, wg, 0, st>>>(__VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t launch_norm2(const BatchHost& bh, int prec, int v_id, int kind, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  STAG_PREC_SWITCH(prec, k_norm2, B, v_id, kind, gate);
  return hipGetLastError();
}

hipError_t launch_update_r(const BatchHost& bh, int prec, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  const int r_id = prec == P64 ? V_R : V_RL;
  STAG_PREC_SWITCH(prec, k_update_r, B, r_id, V_AD);
  return hipGetLastError();
}

hipError_t launch_update_xd(const BatchHost& bh, int prec, int x_prec, int x_id, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  const int r_id = prec == P64 ? V_R : V_RL;
  if (prec == P64 && x_prec == P64)
    k_update_xd<P64, P64><<<nb, wg, 0, st>>>(B, x_id, r_id, V_D);
  else if (prec == P32 && x_prec == P32)
    k_update_xd<P32, P32><<<nb, wg, 0, st>>>(B, x_id, r_id, V_D);
  else if (prec == P16 && x_prec == P32)
    k_update_xd<P16, P32><<<nb, wg, 0, st>>>(B, x_id, r_id, V_D);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_copy_vec(const BatchHost& bh, int src_prec, int src_id, int dst_prec, int dst_id, int gate, int wg,
                           hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
#define STAG_COPY(A, C) \
  if (src_prec == A && dst_prec == C) { k_copy<A, C><<<nb, wg, 0, st>>>(B, src_id, dst_id, gate); return hipGetLastError(); }
  STAG_COPY(P64, P64) STAG_COPY(P64, P32) STAG_COPY(P64, P16) STAG_COPY(P32, P32) STAG_COPY(P16, P16)
  STAG_COPY(P32, P64) STAG_COPY(P16, P64)
#undef STAG_COPY
  return hipErrorInvalidValue;
}

hipError_t launch_rd_dot(const BatchHost& bh, int prec, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  STAG_PREC_SWITCH(prec, k_rd_dot, B, gate);
  return hipGetLastError();
}

hipError_t launch_d_fix(const BatchHost& bh, int prec, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  STAG_PREC_SWITCH(prec, k_d_fix, B, gate);
  return hipGetLastError();
}

hipError_t launch_fcg_dir(const BatchHost& bh, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  k_fcg_dir<<<nb, wg, 0, st>>>(B, gate);
  return hipGetLastError();
}

hipError_t launch_fcg_update(const BatchHost& bh, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  k_fcg_update<<<nb, wg, 0, st>>>(B);
  return hipGetLastError();
}

hipError_t launch_fcg_beta_dot(const BatchHost& bh, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  k_fcg_beta_dot<<<nb, wg, 0, st>>>(B, gate);
  return hipGetLastError();
}

hipError_t launch_add_lo_to_hi(const BatchHost& bh, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  k_add_lo_to_hi<<<nb, wg, 0, st>>>(B, gate);
  return hipGetLastError();
}

hipError_t launch_zero_vec(const BatchHost& bh, int prec, int v_id, int gate, int wg, hipStream_t st) {
  const Batch B = make_batch(bh, wg, 1);
  const int nb = nblocks(B);
  if (nb == 0) return hipSuccess;
  STAG_PREC_SWITCH(prec, k_zero, B, v_id, gate);
  return hipGetLastError();
}

hipError_t launch_finalize(const BatchHost& bh, int what, int kind, int gate, int producer_wg, double* hist,
                           int hist_stride, hipStream_t st, int aux_wg) {
  if (bh.nslots == 0) return hipSuccess;
  const Batch B = make_batch(bh, producer_wg, 1);
  k_finalize<<<bh.nslots, kFinWG, 0, st>>>(B, what, kind, gate, producer_wg, aux_wg > 0 ? aux_wg : producer_wg, hist,
                                        hist_stride);
  return hipGetLastError();
}

// Time-slice sums for the pion correlator of point-source propagators:
//   out[g][t] = (accumulate ? out[g][t] : 0) + weight * sum_{r in group g} sum_{i < slice} |v_r(t * slice + i)|^2
// The sites of one time slice and parity are the contiguous even-odd range [t * slice, (t + 1) * slice).
// One workgroup per (group, slice) sums its slice in a fixed order: the result does not depend on the
// launch.  FP64 colour vectors.
__global__ __launch_bounds__(kMaxWG) void k_slice_norm2(const char* v, long half, int slice, int lt, int group,
                                                        double weight, int accumulate, double* out) {
  __shared__ double lds[4];
  const int t = blockIdx.x % lt, g = blockIdx.x / lt;
  double acc[1] = {0.0};
  for (int r = 0; r < group; ++r) {
    const char* base = v + (long)(g * group + r) * half * spinor_bytes(P64);
    for (int i = threadIdx.x; i < slice; i += blockDim.x) {
      Cx<double> c[3];
      load_spinor<P64, true>(base, (long)t * slice + i, c);
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[0] += c[k].re * c[k].re + c[k].im * c[k].im;
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) {
    const double val = weight * acc[0];
    out[blockIdx.x] = accumulate ? out[blockIdx.x] + val : val;
  }
}

hipError_t launch_slice_norm2(const void* v, long half, int slice, int lt, int ngroups, int group, double weight,
                              int accumulate, double* out, hipStream_t st) {
  if (ngroups == 0) return hipSuccess;
  k_slice_norm2<<<ngroups * lt, kMaxWG, 0, st>>>(reinterpret_cast<const char*>(v), half, slice, lt, group, weight,
                                                 accumulate, out);
  return hipGetLastError();
}

}  // namespace stag
