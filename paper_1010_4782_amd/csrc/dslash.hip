// Even-odd staggered Dslash for gfx950 (Eq. (5) with folded phases plus the
// three-hop Naik term), one output site per lane and R right-hand sides per
// lane so that every link load serves R colour vectors.
//
//   out_p(n) = sum_{k<16} L_k(n) in_{1-p}(n + delta_k),  delta_k in {+-mu, +-3mu}
//
// L_k are the packed, phase-, sign- and c_N-folded matrices (pack.hip).  The
// link stream is the compulsory traffic (16 x 144 B per site in FP64) and is
// read with non-temporal loads; neighbour colour vectors come through L1/L2,
// which the XCD-aware block order keeps local.  With 8 right-hand sides the
// loads of a site's 16 neighbours x R vectors keep the CU's vector-memory
// address and data units nearly always busy, mostly waiting on lines from
// beyond L2: the loads each CU keeps in flight, more than HBM, set the pace.  The output (and the epilogue's
// one read of x or b per site) also goes non-temporal, so that it does not take
// L2 lines from the neighbours: 9% off the FP16 launch inside the CG solve.
#include <algorithm>

#include "device.h"
#include "launch.h"

namespace stag {

// Issue the loads of link k of this lane's site and of the R colour vectors it multiplies (only for the
// active RHS; `on` is uniform over the workgroup).
template <int P, bool C12, int R>
__device__ __forceinline__ void dslash_issue_r(int k, const Site& s, const Geo& g, const char* lbase, long blk,
                                               int lane, const char* in, long rstride_in, const bool on[R],
                                               RawLink<P>& l, RawSpinor<P> v[R]) {
  const int mu = k >> 2, j = k & 3;
  const int nb = neighbour(s, g, mu, j < 2 ? g.h1[mu] : g.h3[mu], (j & 1) == 0);
  const char* slot = lbase + link_slot_offset(P, C12, blk, k);
  if (C12 && j >= 2)
    raw_link_load<P, 2>(slot, lane, l);
  else
    raw_link_load<P, 3>(slot, lane, l);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (on[r]) raw_spinor_load<P>(in + r * rstride_in, nb, v[r]);
}

// The i-th matrix an output site accumulates: f16_link_order for FP16, index order otherwise.
template <int P> __device__ __forceinline__ constexpr int link_at(int i) { return P == P16 ? f16_link_order(i) : i; }

// FP16: acc += (link scale x vector scale) (L v) for one colour vector v of a link L in dot2 form.
template <bool C12>
__device__ __forceinline__ void apply_link_h(const LinkH& L, bool long_link, const RawSpinor<P16>& v, float lsc,
                                             Cx<float> acc[3]) {
  const float s = lsc * __uint_as_float(v.w.w);
  if (C12 && long_link)
    matvec_h_acc<2>(L, v.w.x, v.w.y, v.w.z, s, acc);
  else
    matvec_h_acc<3>(L, v.w.x, v.w.y, v.w.z, s, acc);
}
template <bool C12>
__device__ __forceinline__ void prepare_link_h(const RawLink<P16>& lr, bool long_link, float lsc, float row3,
                                               LinkH& L) {
  if (C12 && long_link)
    link_h_prepare<2>(lr, row3 * lsc, L);
  else
    link_h_prepare<3>(lr, 0.f, L);
}

// Prefetch distance (links) of the single right-hand-side kernel, per storage precision, from a
// sweep of 0-16 on the 28^3x96 lattice: the compiler's own schedule keeps 2-4 loads in flight,
// and these distances are 6% (f16), 8% (f32) and 9% (f64) faster.
template <int P> constexpr int dslash_pf() { return P == P16 ? 12 : (P == P32 ? 8 : 6); }
// With several RHS per lane the link loads are pipelined too, over fewer links, since each stage holds
// R colour vectors in flight.
template <int P, int R> constexpr int dslash_pf_r() {
  if (R == 1) return dslash_pf<P>();
  if (P == P16) return R == 2 ? 8 : (R == 4 ? 4 : 2);
  // FP32 and FP64, measured at 48^3x144 x 8 RHS: 4 and 2 links ahead at R = 4 and 8 (FP64: 7.1 and
  // 5.6 ms per launch against 8.1 and 6.4 ms at 2 and 1, although the deeper pipeline leaves one wave
  // per SIMD at R = 8; FP32: 3.40 and 2.81 ms against 3.46 and 2.91 ms)
  return R == 2 ? 4 : (R == 4 ? 4 : 2);
}

// LDS staging (LDS = true): before the link loop a workgroup copies into LDS the colour vectors of
// the window [c0 - 3 Xh, c0 + wg + 3 Xh) of its first site c0 (for each of its RHS); the x and y
// neighbours of its sites that fall in the window (all but the y neighbours that wrap around the
// lattice) are then read from LDS instead of through L1/L2.  Same arithmetic, same result.
extern __shared__ __align__(16) char dslash_window[];

__host__ __device__ constexpr int window_margin(int xh) { return 3 * xh; }

// Tile order 1 (XCD blocks): the z extent is cut into nzb = 8 c blocks (c = the shape's chunks), c per
// XCD, and the workgroups of an XCD (a contiguous range of positions, xcd_remap) sweep t through one
// block, then the next: the colour vectors of the t +-1, +-3 neighbours of a block's slices are then
// still in that XCD's L2 when they are read again, which the lattice order (t slowest) loses once a slice
// of all RHS outgrows L2.  Thinner blocks keep more of the t window in L2 but read more z neighbours
// (3 planes on each side) from outside the block; the autotuner picks c.  Tiles stay contiguous site
// ranges (a whole number of them per z plane), so every tile is computed exactly as in the lattice
// order; the shape is valid only where that holds (xcd_order_ok).
constexpr int kZBlocks = 8;
__host__ __device__ inline bool xcd_order_ok(int ny, int nz, int xh, int wg, int nzb) {
  return nzb > 0 && nz % nzb == 0 && (ny * xh) % wg == 0;
}
__device__ __forceinline__ int xcd_block_tile(int pos, const Geo& g, int wg, int nzb) {
  const int tpz = g.L[1] * g.Xh / wg;  // tiles per z plane
  const int zbs = g.L[2] / nzb;
  const int j = pos % tpz;
  int rest = pos / tpz;
  const int zi = rest % zbs;
  rest /= zbs;
  const int t = rest % g.L[3];
  const int zb = rest / g.L[3];
  return (t * g.L[2] + zb * zbs + zi) * tpz + j;
}

template <int P, int R, int EPI, bool C12, int PF, bool LDS>
__global__ __launch_bounds__(kMaxWG) void k_dslash(Batch B, int out_par, int in_id, int out_id, int x_id,
                                                   int b_id, int gate, int nzb) {
  static_assert(!(LDS && PF > 0), "the staged path uses the plain link loop");
  using T = typename RealOf<P>::T;
  __shared__ double lds[R * 4];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int p = find_problem(B, bid);
  const ProbDev* pd = B.probs + p;
  const Geo g = pd->g;
  const int local = bid - B.block_start[p];
  const int groups = B.groups[p];
  const int pos = local / groups;
  const int r0 = (local - pos * groups) * R;
  const int nrhs = pd->nrhs, slot0 = pd->slot0;
  const int tile = nzb ? xcd_block_tile(pos, g, blockDim.x, nzb) : pos;  // nzb 0: lattice order

  bool on[R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    on[r] = (r0 + r < nrhs) && slot_on(B.scal, slot0 + r0 + r, gate);
    any |= on[r];
  }
  if (!any) return;  // uniform over the workgroup

  const int cb_raw = tile * blockDim.x + threadIdx.x;
  const bool live = cb_raw < g.half;
  const int cb = live ? cb_raw : g.half - 1;  // dead lanes read a valid site and store nothing
  const Site s = site_of(cb, out_par, g);
  const long gcb = cb + (long)g.t0 * g.stride[3];  // the site's index in the whole lattice: packed links
  const long blk = gcb >> 6;
  const int lane = (int)(gcb & 63);

  const long rstride = (long)g.half * spinor_bytes(P);
  const long rstride_in = (long)g.in_half * spinor_bytes(P);
  const char* in = reinterpret_cast<const char*>(pd->vec[in_id]) + (long)r0 * rstride_in;
  const char* lbase = reinterpret_cast<const char*>(pd->links[P][out_par]);
  const T cn_inv = (T)g.cn_inv;
  // FP16: the matrices stay in code units; each link's scale multiplies the colour vector instead
  float sc_fat = 1.f, sc_long = 1.f;
  if (P == P16) {
    gptr<float> ls = as_global<float>(pd->lscale[out_par]) + blk * 2 * kWave + lane;
    sc_fat = ls[0];
    sc_long = ls[kWave];
  }

  Cx<T> acc[R][3];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = Cx<T>{T(0), T(0)};

  // LDS window: sites [w0, w0 + wn) of every active RHS, 8-byte units, loaded by the whole workgroup
  const int w0 = tile * (int)blockDim.x - window_margin(g.Xh);
  const int wn = (int)blockDim.x + 2 * window_margin(g.Xh);
  constexpr int SB = spinor_bytes(P);
  if constexpr (LDS) {
    const int units = wn * SB / 8;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!on[r]) continue;  // uniform over the workgroup
      // window sites outside [0, in_half) are never read back: every neighbour index is in range
      const char* src = in + r * rstride_in;
      char* dst = dslash_window + r * wn * SB;
      for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int site = w0 + (u * 8) / SB;
        if (site >= 0 && site < g.in_half)
          *reinterpret_cast<u2v*>(dst + u * 8) = *as_global<u2v>(src + (long)w0 * SB + (long)u * 8);
      }
    }
    __syncthreads();
  }

  // The FP16 launches take the 16 matrices in f16_link_order and multiply binary16 codes with dot2
  // (apply_link_h); FP32 and FP64 take them in index order with decoded matrices.  Either way every
  // launch shape of a precision does the same arithmetic in the same order.
  if constexpr (PF > 0) {
    // Software pipeline over the 16 links: the loads of link i + PF are issued while link i is
    // multiplied.  An empty volatile asm that takes the accumulators closes each stage: the
    // products of link i must be done before it and the loads issued after it cannot move above
    // it, so the compiler can neither hoist all loads to the top nor sink them to their uses.
    RawLink<P> lb[PF];
    RawSpinor<P> vb[PF][R];
#pragma unroll
    for (int i = 0; i < PF; ++i)
      dslash_issue_r<P, C12, R>(link_at<P>(i), s, g, lbase, blk, lane, in, rstride_in, on, lb[i], vb[i]);
#pragma unroll
    for (int i = 0; i < kLinks; ++i) {
      const int k = link_at<P>(i);
      const int mu = k >> 2, j = k & 3;
      const float lsc = j < 2 ? sc_fat : sc_long;
      if constexpr (P == P16) {
        LinkH L;
        prepare_link_h<C12>(lb[i % PF], j >= 2, lsc, (float)long_sign(s, g, mu, j == 2) * cn_inv, L);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (on[r]) apply_link_h<C12>(L, j >= 2, vb[i % PF][r], lsc, acc[r]);
      } else {
        Cx<T> u[9];
        if (C12 && j >= 2) {
          raw_link_decode<P, 2>(lb[i % PF], 1.f, u);
          rebuild_row3(u, (T)long_sign(s, g, mu, j == 2) * cn_inv);
        } else {
          raw_link_decode<P, 3>(lb[i % PF], 1.f, u);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!on[r]) continue;
          Cx<T> v[3];
          raw_spinor_decode<P>(vb[i % PF][r], 1.f, v);
          matvec_acc(u, v, acc[r]);
        }
      }
      if (i + PF < kLinks)
        dslash_issue_r<P, C12, R>(link_at<P>(i + PF), s, g, lbase, blk, lane, in, rstride_in, on, lb[i % PF],
                                  vb[i % PF]);
#pragma unroll
      for (int r = 0; r < R; ++r)
        asm volatile("" : "+v"(acc[r][0].re), "+v"(acc[r][0].im), "+v"(acc[r][1].re), "+v"(acc[r][1].im),
                     "+v"(acc[r][2].re), "+v"(acc[r][2].im));
    }
  } else {
#pragma unroll
    for (int i = 0; i < kLinks; ++i) {
      const int k = link_at<P>(i);
      const int mu = k >> 2, j = k & 3;
      const int hop = j < 2 ? g.h1[mu] : g.h3[mu];
      const int nb = neighbour(s, g, mu, hop, (j & 1) == 0);
      const float lsc = j < 2 ? sc_fat : sc_long;
      const bool from_lds = LDS && mu < 2 && (unsigned)(nb - w0) < (unsigned)wn;
      const char* slot = lbase + link_slot_offset(P, C12, blk, k);
      RawLink<P> lr;
      if (C12 && j >= 2)
        raw_link_load<P, 2>(slot, lane, lr);
      else
        raw_link_load<P, 3>(slot, lane, lr);
      RawSpinor<P> vr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!on[r]) continue;
        if (from_lds)
          raw_spinor_lds<P>(dslash_window + r * wn * SB, nb - w0, vr[r]);
        else
          raw_spinor_load<P>(in + r * rstride_in, nb, vr[r]);
      }
      if constexpr (P == P16) {
        LinkH L;
        prepare_link_h<C12>(lr, j >= 2, lsc, (float)long_sign(s, g, mu, j == 2) * cn_inv, L);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (on[r]) apply_link_h<C12>(L, j >= 2, vr[r], lsc, acc[r]);
      } else {
        Cx<T> u[9];
        if (C12 && j >= 2) {
          raw_link_decode<P, 2>(lr, 1.f, u);
          rebuild_row3(u, (T)long_sign(s, g, mu, j == 2) * cn_inv);
        } else {
          raw_link_decode<P, 3>(lr, 1.f, u);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!on[r]) continue;
          Cx<T> v[3];
          raw_spinor_decode<P>(vr[r], 1.f, v);
          matvec_acc(u, v, acc[r]);
        }
      }
    }
  }

  char* out = reinterpret_cast<char*>(pd->vec[out_id]) + (long)r0 * rstride;
  if (EPI == EPI_PLAIN) {
    if (live)
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (on[r]) store_spinor<P, true, true>(out + r * rstride, cb, acc[r]);
    return;
  }

  const char* xb = reinterpret_cast<const char*>(pd->vec[x_id]) + (long)r0 * rstride;
  double part[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    part[r] = 0.0;
    if (!on[r]) continue;
    const T a = (T)B.scal[slot0 + r0 + r].mass4;
    Cx<T> xv[3], o[3];
    load_spinor<P, true>(xb + r * rstride, cb, xv);
    if (EPI == EPI_RESID) {
      Cx<T> bv[3];
      load_spinor<P, true>(reinterpret_cast<const char*>(pd->vec[b_id]) + (long)(r0 + r) * rstride, cb, bv);
#pragma unroll
      for (int c = 0; c < 3; ++c)
        o[c] = Cx<T>{bv[c].re - a * xv[c].re + acc[r][c].re, bv[c].im - a * xv[c].im + acc[r][c].im};
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) o[c] = Cx<T>{a * xv[c].re - acc[r][c].re, a * xv[c].im - acc[r][c].im};
    }
    if (live) {
      store_spinor<P, true, true>(out + r * rstride, cb, o);
      if (EPI == EPI_XPAY_DOT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) part[r] += (double)xv[c].re * (double)o[c].re + (double)xv[c].im * (double)o[c].im;
      } else if (EPI == EPI_RESID) {
#pragma unroll
        for (int c = 0; c < 3; ++c) part[r] += (double)o[c].re * (double)o[c].re + (double)o[c].im * (double)o[c].im;
      }
    }
  }
  if (EPI == EPI_XPAY) return;
  block_sum<R>(part, lds);
  if (threadIdx.x == 0) {
    const int kind = EPI == EPI_XPAY_DOT ? 0 : 1;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (on[r]) B.partial[((long)(slot0 + r0 + r) * kPartialSlots + kind) * B.pstride + tile] = part[r];
  }
}

Batch make_batch(const BatchHost& bh, int wg, int r) {
  Batch B{};
  B.probs = bh.d_probs;
  B.scal = bh.d_scal;
  B.partial = bh.d_partial;
  B.pstride = bh.pstride;
  B.nprob = (int)bh.probs.size();
  B.block_start[0] = 0;
  for (int p = 0; p < B.nprob; ++p) {
    B.tiles[p] = ceil_div(bh.probs[p].half, wg);
    B.groups[p] = ceil_div(bh.probs[p].nrhs, r);
    B.block_start[p + 1] = B.block_start[p] + B.tiles[p] * B.groups[p];
  }
  return B;
}

template <int P, int R, bool C12, bool LDS>
static hipError_t dslash_r(const Batch& B, int nblk, int epi, int out_par, int in_id, int out_id, int x_id, int b_id,
                           int gate, int wg, int order, size_t lds_bytes, hipStream_t st) {
  constexpr int PF = !LDS ? dslash_pf_r<P, R>() : 0;
  constexpr int PF64 = !LDS ? dslash_pf_r<P64, R>() : 0;
  switch (epi) {
    case EPI_PLAIN:
      k_dslash<P, R, EPI_PLAIN, C12, PF, LDS><<<nblk, wg, lds_bytes, st>>>(B, out_par, in_id, out_id, x_id, b_id, gate, order);
      break;
    case EPI_XPAY_DOT:
      k_dslash<P, R, EPI_XPAY_DOT, C12, PF, LDS><<<nblk, wg, lds_bytes, st>>>(B, out_par, in_id, out_id, x_id, b_id,
                                                                            gate, order);
      break;
    case EPI_RESID:
      if (P != P64) return hipErrorInvalidValue;
      k_dslash<P64, R, EPI_RESID, C12, PF64, LDS><<<nblk, wg, lds_bytes, st>>>(B, out_par, in_id, out_id, x_id, b_id,
                                                                             gate, order);
      break;
    case EPI_XPAY:
      if (P != P64) return hipErrorInvalidValue;
      k_dslash<P64, R, EPI_XPAY, C12, PF64, LDS><<<nblk, wg, lds_bytes, st>>>(B, out_par, in_id, out_id, x_id, b_id,
                                                                            gate, order);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P, bool C12, bool LDS>
static hipError_t dslash_p(const Batch& B, int nblk, int epi, int out_par, int in_id, int out_id, int x_id, int b_id,
                           int gate, int wg, int r, int order, size_t lds_bytes, hipStream_t st) {
  switch (r) {
    case 1: return dslash_r<P, 1, C12, LDS>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, wg, order, lds_bytes, st);
    case 2: return dslash_r<P, 2, C12, LDS>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, wg, order, lds_bytes, st);
    case 4: return dslash_r<P, 4, C12, LDS>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, wg, order, lds_bytes, st);
    case 8: return dslash_r<P, 8, C12, LDS>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, wg, order, lds_bytes, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t dslash_pc(const Batch& B, int nblk, int epi, int out_par, int in_id, int out_id, int x_id, int b_id,
                            int gate, const DslashShape& sh, bool c12, size_t lds_bytes, hipStream_t st) {
  const int nzb = sh.order == 1 ? kZBlocks * sh.chunks : 0;  // z blocks of the XCD order, 0: lattice order
  if (c12)
    return sh.lds ? dslash_p<P, true, true>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh.wg, sh.r,
                                            nzb, lds_bytes, st)
                  : dslash_p<P, true, false>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh.wg, sh.r,
                                             nzb, 0, st);
  return sh.lds ? dslash_p<P, false, true>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh.wg, sh.r,
                                           nzb, lds_bytes, st)
                : dslash_p<P, false, false>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh.wg, sh.r,
                                            nzb, 0, st);
}

// The LDS window holds wg + 6 Xh sites (of the widest lattice of the batch) per RHS of a lane.
size_t dslash_lds_bytes(const BatchHost& bh, int prec, const DslashShape& sh) {
  if (!sh.lds) return 0;
  int xh = 0;
  for (const auto& p : bh.probs) xh = std::max(xh, p.xh);
  return (size_t)sh.r * (sh.wg + 2 * window_margin(xh)) * spinor_bytes(prec);
}

bool dslash_shape_valid(const BatchHost& bh, int prec, const DslashShape& sh) {
  if (sh.order == 2) return prec == P16 && sh.wg == 64 && sh.lds == 0 && dslash_t_ok(bh, sh.r, sh.chunks);
  if (sh.wg != 64 && sh.wg != 128 && sh.wg != 256) return false;
  if (sh.r != 1 && sh.r != 2 && sh.r != 4 && sh.r != 8) return false;
  if (sh.order != 0 && sh.order != 1) return false;
  if (sh.order == 0 && sh.chunks != 1) return false;
  if (sh.order)
    for (const auto& p : bh.probs)
      if (!xcd_order_ok(p.ny, p.nz, p.xh, sh.wg, kZBlocks * sh.chunks)) return false;
  return dslash_lds_bytes(bh, prec, sh) <= kMaxDslashLds;
}

hipError_t launch_dslash(const BatchHost& bh, int prec, int epi, int out_par, int in_id, int out_id, int x_id,
                         int b_id, int gate, const DslashShape& sh, hipStream_t st) {
  if (!dslash_shape_valid(bh, prec, sh)) return hipErrorInvalidValue;
  if (sh.order == 2) return launch_dslash_t(bh, epi, out_par, in_id, out_id, x_id, gate, sh.r, sh.chunks, st);
  const Batch B = make_batch(bh, sh.wg, sh.r);
  const int nblk = B.block_start[B.nprob];
  if (nblk == 0) return hipSuccess;
  const bool c12 = bh.long12;
  const size_t lds = dslash_lds_bytes(bh, prec, sh);
  switch (prec) {
    case P64: return dslash_pc<P64>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh, c12, lds, st);
    case P32: return dslash_pc<P32>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh, c12, lds, st);
    case P16: return dslash_pc<P16>(B, nblk, epi, out_par, in_id, out_id, x_id, b_id, gate, sh, c12, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace stag
