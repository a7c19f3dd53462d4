// Internal types shared by the host runtime and the HIP kernels of libstagcg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stag {

constexpr int kWave = 64;        // gfx950 wavefront
constexpr int kMaxWG = 256;      // largest workgroup any kernel is launched with
constexpr int kLinks = 16;       // packed matrices per output site: 4 directions x {fat fwd, fat bwd, long fwd, long bwd}
constexpr int kMaxProb = 16;     // problems per batched launch
constexpr int kPartialSlots = 3; // reduction partials per slot kept apart (up to three sums)

enum Prec : int { P64 = 0, P32 = 1, P16 = 2 };

// Storage of one packed link per lane: 9 complex numbers, or 6 (two rows) for a three-hop link stored
// with 12 real parameters (its third row is rebuilt from the first two; SU(3) links only).
__host__ __device__ constexpr int link_bytes(int p) { return p == P64 ? 144 : (p == P32 ? 72 : 36); }
__host__ __device__ constexpr int link12_bytes(int p) { return p == P64 ? 96 : (p == P32 ? 48 : 24); }

// Packed links of one output parity, per block of 64 output sites: eight one-hop slots (k = 4 mu + j,
// j = 0 forward, 1 backward -> slot 2 mu + j) of link_bytes(P) per lane, then eight three-hop slots
// (j = 2, 3 -> slot 2 mu + j - 2) of link_bytes(P) or, compressed, link12_bytes(P) per lane.
__host__ __device__ constexpr long link_block_bytes(int p, bool c12) {
  return 64L * 8 * (link_bytes(p) + (c12 ? link12_bytes(p) : link_bytes(p)));
}
__host__ __device__ inline long link_slot_offset(int p, bool c12, long blk, int k) {
  const int mu = k >> 2, j = k & 3;
  const long b = blk * link_block_bytes(p, c12);
  if (j < 2) return b + (long)(2 * mu + j) * 64 * link_bytes(p);
  return b + 64L * 8 * link_bytes(p) + (long)(2 * mu + j - 2) * 64 * (c12 ? link12_bytes(p) : link_bytes(p));
}
// Storage of one colour vector (3 complex) per site.  f16: six binary16 codes + one binary32 scale.
__host__ __device__ constexpr int spinor_bytes(int p) { return p == P64 ? 48 : (p == P32 ? 24 : 16); }

// Lattice geometry in the even-odd index cb = lex >> 1.
struct Geo {
  int L[4];        // Lx, Ly, Lz, Lt
  int antiper;     // 1: antiperiodic time direction
  int long12;      // 1: three-hop links stored with 12 real parameters
  double cn_inv;   // 1 / c_N (rebuilding the third row of a compressed three-hop link)
  int Xh;          // Lx / 2
  int half;        // V / 2
  int stride[4];   // cb distance of one step in y, z, t (stride[0] unused: x is handled by parity)
  int h1[4];       // 1 mod L_mu
  int h3[4];       // 3 mod L_mu
  // A time slab [t0, t0 + L[3]) of a lattice with lt_glob slices (domain decomposition along t):
  // t_open = 1 stops the time neighbours from wrapping; they are read from 3 ghost slices on each
  // side of the input field, which then holds in_half = (L[3] + 6) * stride[3] sites per RHS.
  // A whole lattice has t0 = 0, lt_glob = L[3], t_open = 0, in_half = half.
  int t0;
  int lt_glob;
  int h3g;         // 3 mod lt_glob
  int t_open;
  int in_half;
};

// Per right-hand-side solver state ("slot"), resident on the device.
// state: 0 running, 1 stopped in this iteration (x update still pending), 2 stopped,
//        3 finished (excluded from every stage until the host restarts it).
struct Scal {
  double b2;         // ||b||^2
  double thr;        // stopping threshold on r^dag r
  double delta;      // r^dag r (current)
  double delta_old;
  double dAd;        // Re d^dag A d
  double alpha;
  double beta;
  double mass4;      // 4 m^2
  double rz;         // FCG: <z, r>
  double rz_new;     // FCG
  double aux;        // scratch scalar (true residual, stall monitor)
  double rel_thr;    // mixed precision: r^dag r below which a reliable update is due
  double cre, cim;   // mixed precision: d += (cre + i cim) r after a reliable update
  double ar, ai;     // flexible CG: complex alpha = <d, r> / <d, A d>
  double br, bi;     // flexible CG: complex beta = -<A d_prev, z> / <d_prev, A d_prev>
  double dmin;       // flexible CG: smallest r^dag r seen (the stall test compares it window to window)
  int state;
  int iter;          // iterations since the last (re)start
  int max_iter;
  int flags;         // bit 0: NaN / breakdown, bit 1: hit max_iter
  int hist_len;      // number of (alpha, beta) pairs to record
  int pad[3];
};
static_assert(sizeof(Scal) % 8 == 0, "Scal alignment");

enum ScalFlags : int { kFlagNaN = 1, kFlagMaxIter = 2, kFlagRelDue = 4, kFlagBreakdown = 8 };

// Vector roles in a solver workspace (one [nrhs][V/2][3] array per role and problem).
enum VecId : int {
  V_B = 0,     // f64 source (caller's)
  V_X,         // f64 solution (caller's)
  V_R,         // f64 residual
  V_D,         // search direction (inner precision)
  V_AD,        // A d (inner precision)
  V_T,         // odd-parity temporary (inner precision)
  V_RL,        // low-precision residual (mixed precision)
  V_XL,        // f32 low-precision solution accumulator (mixed precision)
  V_TMP,       // f64 even temporary
  V_TMPO,      // f64 odd temporary
  V_Z,         // FCG: preconditioned residual
  V_RPREV,     // FCG: previous residual
  V_NETA,      // network activations
  V_NETB,
  kNumVec
};

// One problem as the kernels see it.
struct ProbDev {
  Geo g;
  const void* links[3][2];  // packed links per storage precision and output parity (null if not built)
  const float* lscale[2];   // f16 link-group scales per output parity (null if not built)
  void* vec[kNumVec];
  int nrhs;
  int slot0;                // first scalar slot of this problem
  int pad[2];
};

// Arguments of a batched launch: problems and where each starts in the block space.
struct Batch {
  const ProbDev* probs;     // device table
  Scal* scal;               // device [nslots]
  double* partial;          // device [nslots][kPartialSlots][pstride]
  int pstride;              // partial entries per slot and kind
  int nprob;
  int block_start[kMaxProb + 1];
  int tiles[kMaxProb];      // site tiles per RHS group
  int groups[kMaxProb];     // RHS groups per problem
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace stag
