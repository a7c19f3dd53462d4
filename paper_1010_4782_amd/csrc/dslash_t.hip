// Time-streaming FP16 Dslash for many right-hand sides (Eq. (5) with folded phases plus the three-hop
// Naik term; the same sum as k_dslash, in the same order, so the same bits).
//
// With 8 right-hand sides a time slice of binary16 colour vectors is 128 B per site, and the t +-1, +-3
// neighbours of the site-parallel kernel are read again one to three slices later, by when an XCD's
// 4 MB L2 no longer holds them: the input is fetched about four times.  Here a wave owns 64 sites of the
// slice plane (one lane per site, eight RHS per lane) and one class of time slices (t even or t odd) and
// walks t.  At every step it loads the input slice s at its own sites once and hands it to the four
// outputs that need it as a time neighbour (s -+ 1, s -+ 3, all of the wave's class), while the waves of
// the other class read the same slice, at the same step, as the x/y/z neighbours of their outputs at s:
// every slice is consumed in the step it arrives, and the L2 only has to hold about one slice of the
// XCD's share of the plane.  An output therefore collects its matrices over seven steps
//     t-3: k=15 (-3t)   t-1: k=13 (-1t)   t: k=0..11 (x, y, z)   t+1: k=12 (+1t)   t+3: k=14 (+3t)
// f16_link_order is exactly this order.  One iteration of the loop is one spatial step and one
// time-hop step: 16 link applications.  The link of application a + 2 is requested while a is
// multiplied, and each right-hand side's vectors for the next application as soon as that RHS is done
// with the current one.  The output of the spatial step (13 of its 16 matrices arrive in this
// iteration) is accumulated in registers; the three outputs that take one matrix each (t - 2, t + 2,
// t + 4) wait in LDS, in a ring of three entries, so that the wave fits in 256 VGPRs.  The reduction
// partial of the xpay epilogue covers the same 64 sites, in the same order, as a 64-site workgroup of
// the site-parallel kernel, so the whole CG iteration gives the same bits with either kernel.
#include "device.h"
#include "launch.h"

namespace stag {

namespace {

constexpr int kTGroup = 8;  // right-hand sides per site of one wave (a lane takes R of them)
constexpr int kTPfL = 2;    // links in flight ahead of the application being multiplied (divides 16)
constexpr int kTHopAt = 10; // application whose RHS loop requests the time-hop input (used by 12..15)
constexpr int kXAt = 11;    // application whose RHS loop requests the xpay epilogue's x (used at 12)

// Application a (0..15) of an iteration: 0..11 spatial matrices k = a of the output in slot 1,
// 12..15 the time hops (k = 14, 12, 13, 15) of the outputs in slots 0..3, all with the input at t + 1.
__device__ __forceinline__ constexpr int app_link(int a) { return a < 12 ? a : (a == 12 ? 14 : (a == 13 ? 12 : (a == 14 ? 13 : 15))); }
__device__ __forceinline__ constexpr int app_slot(int a) { return a < 12 ? 1 : a - 12; }

struct TLane {
  int i;        // in-plane even-odd index of the lane's sites (the same in every slice)
  int S;        // sites of one slice and parity
  int lt;       // time extent
  int ta, tb;   // the wave's chunk of output slices [ta, tb)
  int cls;      // time parity of its outputs
  Site s0;      // the lane's output site in its first slice (x, y, z are those of every slice)
  int eta3;     // (x + y + z) & 1: eta_t of the lane's sites
};

__device__ __forceinline__ int wrap_t(int t, int lt) { t %= lt; return t < 0 ? t + lt : t; }

// folded-scalar sign of the time three-hop matrix (fwd: k = 14, else k = 15) of output slice t
__device__ __forceinline__ int t_long_sign(const TLane& L, const Geo& g, int t, bool fwd) {
  int neg = L.eta3 ^ (fwd ? 0 : 1);
  const int start = fwd ? t : wrap_t(t - 3, g.L[3]);
  const int wraps = (start + 3 >= g.L[3]) ^ (start + 3 >= 2 * g.L[3]);
  neg ^= wraps & g.antiper;
  return neg ? -1 : 1;
}

}  // namespace

// R right-hand sides per lane: LPS = 8 / R lanes share a site (and load its links together), a wave
// covers W = 64 / LPS sites.
template <int R, int EPI, bool C12>
__global__ __launch_bounds__(kWave) void k_dslash_t(Batch B, int out_par, int in_id, int out_id, int x_id, int gate,
                                                    int chunks) {
  constexpr int kTRhs = R;
  constexpr int LPS = kTGroup / R;
  constexpr int W = kWave / LPS;
  // outputs waiting for their time-hop matrices: ring[entry][accumulator][lane]
  __shared__ Cx<float> ring[3][3 * R][kWave];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int p = find_problem(B, bid);
  const ProbDev* pd = B.probs + p;
  const Geo g = pd->g;
  TLane L;
  L.S = g.stride[3];
  L.lt = g.L[3];
  const int ntile = L.S / W;
  const int local = bid - B.block_start[p];
  const int grp = local / B.tiles[p];
  int item = local - grp * B.tiles[p];
  L.cls = item & 1;
  item >>= 1;
  const int tile = item % ntile;
  const int chunk = item / ntile;
  const int lane = threadIdx.x;
  const int hf = lane % LPS;                // which R of the site's 8 RHS
  const int rb = grp * kTGroup + hf * R;    // first RHS of the lane
  const int slot0 = pd->slot0;
  bool on[kTRhs];
  bool any = false;
#pragma unroll
  for (int r = 0; r < kTRhs; ++r) {
    on[r] = slot_on(B.scal, slot0 + rb + r, gate);
    any |= on[r];
  }
  if (!__any(any)) return;  // every RHS of the wave has stopped (uniform)

  const int clen = L.lt / chunks;
  L.ta = chunk * clen;
  L.tb = L.ta + clen;
  L.i = tile * W + lane / LPS;
  L.s0 = site_of(L.i + (L.ta + L.cls) * L.S, out_par, g);
  L.eta3 = (L.s0.x + L.s0.y + L.s0.z) & 1;

  const long rstride = (long)g.half * spinor_bytes(P16);
  const char* in = reinterpret_cast<const char*>(pd->vec[in_id]) + (long)rb * rstride;
  char* out = reinterpret_cast<char*>(pd->vec[out_id]) + (long)rb * rstride;
  const char* xb = reinterpret_cast<const char*>(pd->vec[x_id]) + (long)rb * rstride;
  const char* lbase = reinterpret_cast<const char*>(pd->links[P16][out_par]);
  const float* lscale = pd->lscale[out_par];
  const float cn_inv = (float)g.cn_inv;

  const int t_first = L.ta + L.cls;      // first output of the wave
  const int t_last = L.tb - 2 + L.cls;   // last output
  auto valid = [&](int t) { return t >= t_first && t <= t_last; };
  auto entry = [&](int t) { return ((t - t_first + 6) >> 1) % 3; };  // ring entry of output t (t >= t_first - 6)
  auto load_scales = [&](int t, float& f, float& l) {
    const long gcb = L.i + (long)t * L.S;
    gptr<float> ls = as_global<float>(lscale) + (gcb >> 6) * 2 * kWave + (gcb & 63);
    f = ls[0];
    l = ls[kWave];
  };
  // the link of application a of the iteration with spatial output t
  auto issue_link = [&](int a, int t, RawLink<P16>& lr) {
    const int to = t - 2 + 2 * app_slot(a);  // output slice of the application
    if (!valid(to)) return;
    const int k = app_link(a);
    const long gcb = L.i + (long)to * L.S;
    const char* slot = lbase + link_slot_offset(P16, C12, gcb >> 6, k);
    if (C12 && (k & 3) >= 2)
      raw_link_load<P16, 2>(slot, (int)(gcb & 63), lr);
    else
      raw_link_load<P16, 3>(slot, (int)(gcb & 63), lr);
  };
  // RHS r's x/y/z neighbour k = a (a < 12) of the lane's output site at slice t
  auto issue_vec = [&](int a, int t, int r, RawSpinor<P16>& v) {
    if (!valid(t)) return;
    const int mu = a >> 2, j = a & 3;
    const int off = neighbour(L.s0, g, mu, j < 2 ? g.h1[mu] : g.h3[mu], (j & 1) == 0) - L.s0.cb;
    raw_spinor_load<P16>(in + r * rstride, L.i + (long)t * L.S + off, v);
  };
  auto prepare = [&](int a, int to, float lsc, const RawLink<P16>& lr, LinkH& lh) {
    const int k = app_link(a);
    const int mu = k >> 2, j = k & 3;
    const float row3 =
        (mu < 3 ? (float)long_sign(L.s0, g, mu, j == 2) : (float)t_long_sign(L, g, to, j == 2)) * cn_inv;
    if (C12 && j >= 2)
      link_h_prepare<2>(lr, row3 * lsc, lh);
    else
      link_h_prepare<3>(lr, 0.f, lh);
  };
  auto mul = [&](int a, const LinkH& lh, float lsc, const RawSpinor<P16>& v, Cx<float> acc[3]) {
    const float sv = lsc * __uint_as_float(v.w.w);
    if (C12 && (app_link(a) & 3) >= 2)
      matvec_h_acc<2>(lh, v.w.x, v.w.y, v.w.z, sv, acc);
    else
      matvec_h_acc<3>(lh, v.w.x, v.w.y, v.w.z, sv, acc);
  };

  Cx<float> hot[kTRhs][3];            // the output t of the current iteration
  float h_fat = 0.f, h_long = 0.f;    // its link scales
  RawLink<P16> lb[kTPfL];
  RawSpinor<P16> vb[kTRhs];           // RHS r's vector for the next spatial application
  RawSpinor<P16> vt[kTRhs];           // the input at t + 1 (time hops 12..15)
  RawSpinor<P16> xr[kTRhs];           // xpay: x at the output completed in this iteration
  int t = t_first - 4;  // the first iteration only has the -3 hop of the first output
#pragma unroll
  for (int a = 0; a < kTPfL; ++a) issue_link(a, t, lb[a]);
#pragma unroll
  for (int r = 0; r < kTRhs; ++r) issue_vec(0, t, r, vb[r]);
#pragma unroll 1
  for (; t <= t_last + 2; t += 2) {
    const bool vt_ok = valid(t);
    if (vt_ok) load_scales(t, h_fat, h_long);
#pragma unroll
    for (int r = 0; r < kTRhs; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) hot[r][c] = vt_ok ? ring[entry(t)][3 * r + c][lane] : Cx<float>{0.f, 0.f};
#pragma clang loop unroll(full)
    for (int a = 0; a < 16; ++a) {
      const int to = t - 2 + 2 * app_slot(a);
      const int k = app_link(a);
      const bool ok = valid(to);
      float lsc = (k & 3) >= 2 ? h_long : h_fat;
      float sf = 0.f, sl = 0.f;
      if (ok && a != 13 && a >= 12) {
        load_scales(to, sf, sl);
        lsc = a == 14 ? sf : sl;
      }
      LinkH lh;
      if (ok) prepare(a, to, lsc, lb[a % kTPfL], lh);
      // the link of application a + kTPfL (of this or the next iteration) into the registers just read
      if (a + kTPfL < 16)
        issue_link(a + kTPfL, t, lb[a % kTPfL]);
      else
        issue_link(a + kTPfL - 16, t + 2, lb[a % kTPfL]);
      double part[kTRhs];
#pragma unroll
      for (int r = 0; r < kTRhs; ++r) {
        part[r] = 0.0;
        if (a < 12) {
          if (ok) mul(a, lh, lsc, vb[r], hot[r]);
          // RHS r's vector for the next spatial application (the next iteration's first after a = 11)
          if (a < 11)
            issue_vec(a + 1, t, r, vb[r]);
          else
            issue_vec(0, t + 2, r, vb[r]);
          if (a == kTHopAt) raw_spinor_load<P16>(in + r * rstride, L.i + (long)wrap_t(t + 1, L.lt) * L.S, vt[r]);
          if (EPI == EPI_XPAY_DOT && a == kXAt && valid(t - 2))
            xr[r].w = __builtin_nontemporal_load(as_global<u4v>(xb + r * rstride) + L.i + (long)(t - 2) * L.S);
          asm volatile("" : "+v"(hot[r][0].re), "+v"(hot[r][0].im), "+v"(hot[r][1].re), "+v"(hot[r][1].im),
                       "+v"(hot[r][2].re), "+v"(hot[r][2].im));
        } else if (a == 13) {
          if (ok) mul(a, lh, lsc, vt[r], hot[r]);  // +1 time hop of output t
        } else if (ok) {
          // one matrix for an output waiting in LDS: t - 2 (+3 hop, its last), t + 2 (-1 hop), t + 4
          // (-3 hop, its first)
          const int e = entry(to);
          Cx<float> c[3];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) c[cc] = a == 15 ? Cx<float>{0.f, 0.f} : ring[e][3 * r + cc][lane];
          mul(a, lh, lsc, vt[r], c);
          if (a != 12) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) ring[e][3 * r + cc][lane] = c[cc];
          } else {
            // output t - 2 is complete
            const long cb = L.i + (long)to * L.S;
            if (EPI == EPI_PLAIN) {
              if (on[r]) store_spinor<P16, true, true>(out + r * rstride, cb, c);
            } else if (on[r]) {
              const float a4 = (float)B.scal[slot0 + rb + r].mass4;
              const float xs = __uint_as_float(xr[r].w.w);
              const Cx<float> xv[3] = {unpack_h2(xr[r].w.x, xs), unpack_h2(xr[r].w.y, xs), unpack_h2(xr[r].w.z, xs)};
              Cx<float> o[3];
#pragma unroll
              for (int cc = 0; cc < 3; ++cc)
                o[cc] = Cx<float>{a4 * xv[cc].re - c[cc].re, a4 * xv[cc].im - c[cc].im};
              store_spinor<P16, true, true>(out + r * rstride, cb, o);
#pragma unroll
              for (int cc = 0; cc < 3; ++cc)
                part[r] += (double)xv[cc].re * (double)o[cc].re + (double)xv[cc].im * (double)o[cc].im;
            }
          }
        }
      }
      if (EPI == EPI_XPAY_DOT && a == 12 && ok) {
        // the partials of the W sites of output slice t - 2; with one lane per site exactly as block_sum
        // of a 64-site workgroup of the site-parallel kernel sums them
        if constexpr (LPS == 1) {
          wave_sum<kTRhs>(part);
        } else {
#pragma unroll
          for (int off = kWave / 2; off >= LPS; off >>= 1)
#pragma unroll
            for (int r = 0; r < kTRhs; ++r) part[r] += __shfl_xor(part[r], off, kWave);
        }
        if (lane < LPS) {
          const long tix = (L.i + (long)to * L.S) / W;
#pragma unroll
          for (int r = 0; r < kTRhs; ++r)
            if (on[r]) B.partial[((long)(slot0 + rb + r) * kPartialSlots + 0) * B.pstride + tix] = part[r];
        }
      }
    }
    // output t waits in its ring entry for its +3 time hop (next iteration)
    if (vt_ok)
#pragma unroll
      for (int r = 0; r < kTRhs; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) ring[entry(t)][3 * r + c][lane] = hot[r][c];
  }
}

bool dslash_t_ok(const BatchHost& bh, int r, int chunks) {
  if (chunks < 1 || (r != 4 && r != 8)) return false;
  const int W = kWave / (kTGroup / r);
  for (const auto& p : bh.probs) {
    if (p.t_open || p.nrhs % kTGroup || p.lt % (2 * chunks)) return false;
    const long S = (long)p.half / p.lt;
    if (S % W) return false;
  }
  return true;
}

Batch make_batch_t(const BatchHost& bh, int r, int chunks) {
  const int W = kWave / (kTGroup / r);
  Batch B{};
  B.probs = bh.d_probs;
  B.scal = bh.d_scal;
  B.partial = bh.d_partial;
  B.pstride = bh.pstride;
  B.nprob = (int)bh.probs.size();
  B.block_start[0] = 0;
  for (int p = 0; p < B.nprob; ++p) {
    const int S = bh.probs[p].half / bh.probs[p].lt;
    B.tiles[p] = 2 * (S / W) * chunks;       // work items per group of 8 RHS
    B.groups[p] = bh.probs[p].nrhs / kTGroup;
    B.block_start[p + 1] = B.block_start[p] + B.tiles[p] * B.groups[p];
  }
  return B;
}

template <int R>
static hipError_t launch_t(const Batch& B, int nblk, bool c12, int epi, int out_par, int in_id, int out_id, int x_id,
                           int gate, int chunks, hipStream_t st) {
  switch (epi) {
    case EPI_PLAIN:
      if (c12)
        k_dslash_t<R, EPI_PLAIN, true><<<nblk, kWave, 0, st>>>(B, out_par, in_id, out_id, x_id, gate, chunks);
      else
        k_dslash_t<R, EPI_PLAIN, false><<<nblk, kWave, 0, st>>>(B, out_par, in_id, out_id, x_id, gate, chunks);
      break;
    case EPI_XPAY_DOT:
      if (c12)
        k_dslash_t<R, EPI_XPAY_DOT, true><<<nblk, kWave, 0, st>>>(B, out_par, in_id, out_id, x_id, gate, chunks);
      else
        k_dslash_t<R, EPI_XPAY_DOT, false><<<nblk, kWave, 0, st>>>(B, out_par, in_id, out_id, x_id, gate, chunks);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dslash_t(const BatchHost& bh, int epi, int out_par, int in_id, int out_id, int x_id, int gate,
                           int r, int chunks, hipStream_t st) {
  if (!dslash_t_ok(bh, r, chunks)) return hipErrorInvalidValue;
  const Batch B = make_batch_t(bh, r, chunks);
  const int nblk = B.block_start[B.nprob];
  if (nblk == 0) return hipSuccess;
  return r == 8 ? launch_t<8>(B, nblk, bh.long12, epi, out_par, in_id, out_id, x_id, gate, chunks, st)
                : launch_t<4>(B, nblk, bh.long12, epi, out_par, in_id, out_id, x_id, gate, chunks, st);
}

}  // namespace stag
