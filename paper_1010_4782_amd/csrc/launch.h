// Host-side launchers of the HIP kernels (declared here, defined in the .hip files).
#pragma once

#include <vector>

#include "stag_internal.h"

namespace stag {

enum Epi : int {
  EPI_PLAIN = 0,     // out = D in
  EPI_XPAY_DOT = 1,  // out = 4m^2 x - D in ; partial[kind 0] = Re <x, out>
  EPI_RESID = 2,     // out = b - (4m^2 x - D in) ; partial[kind 1] = |out|^2   (FP64 only)
  EPI_XPAY = 3       // out = 4m^2 x - D in                                      (FP64 only)
};

// Host mirror of a batch: sizes the launchers need to build the block map.
struct HostProb {
  int half;
  int nrhs;
  int slot0;
  int xh = 0;  // Lx / 2 (width of the LDS window margin of a staged Dslash)
  int ny = 0, nz = 0;  // Ly, Lz (whether the XCD-block tile order fits the lattice)
  int lt = 0;          // Lt (of the slab, for a slab launch)
  int t_open = 0;      // 1: a time slab with ghost slices (stag_dslash_slab)
};

constexpr int kTGroupRhs = 8;  // right-hand sides per site of a time-streaming wave

constexpr size_t kMaxDslashLds = 64 * 1024;  // LDS a staged Dslash workgroup may use

struct BatchHost {
  std::vector<HostProb> probs;
  const ProbDev* d_probs = nullptr;
  Scal* d_scal = nullptr;
  double* d_partial = nullptr;
  int pstride = 0;
  int nslots = 0;
  int max_half = 0;
  bool long12 = false;   // every lattice of the batch stores its three-hop links as two rows
};

// Block map for a launch with `wg` sites per workgroup and `r` right-hand sides per lane.
Batch make_batch(const BatchHost& bh, int wg, int r);

// Launch shape of a Dslash: sites per workgroup, right-hand sides per lane, LDS staging.
struct DslashShape {
  int wg = 256;
  int r = 1;
  int lds = 0;  // 1: stage the x and y neighbour colour vectors of a workgroup's sites in LDS
  int order = 0;  // 1: XCD-block tile order (each XCD sweeps t through one z block);
                  // 2: the time-streaming FP16 kernel (dslash_t.hip): wg 64 (one wave), r 8 (one lane per
                  //    site) or r 4 (two lanes per site, 32 sites per wave)
  int chunks = 1; // order 2: the time extent is walked in this many chunks (one wave per chunk)
};

// Sites per reduction partial of the xpay launch of this shape (the finalize's producer_wg).
inline int partial_wg(const DslashShape& s) { return s.order == 2 ? s.wg / (kTGroupRhs / s.r) : s.wg; }

// Bytes of LDS a staged launch of this shape needs (0 if unstaged), and whether it fits.
size_t dslash_lds_bytes(const BatchHost& bh, int prec, const DslashShape& sh);
bool dslash_shape_valid(const BatchHost& bh, int prec, const DslashShape& sh);
hipError_t launch_dslash(const BatchHost& bh, int prec, int epi, int out_par, int in_id, int out_id, int x_id,
                         int b_id, int gate, const DslashShape& sh, hipStream_t st);
// The time-streaming FP16 kernel (plain or xpay + <d, Ad> epilogue) and whether a batch fits it.
bool dslash_t_ok(const BatchHost& bh, int r, int chunks);
hipError_t launch_dslash_t(const BatchHost& bh, int epi, int out_par, int in_id, int out_id, int x_id, int gate,
                           int r, int chunks, hipStream_t st);

// Vector stages of the solvers (every one is one launch over all slots of the batch).
hipError_t launch_norm2(const BatchHost& bh, int prec, int v_id, int kind, int gate, int wg, hipStream_t st);
hipError_t launch_slice_norm2(const void* v, long half, int slice, int lt, int ngroups, int group, double weight,
                              int accumulate, double* out, hipStream_t st);
// producer_wg: sites per block of the launch that wrote the first partial kind; aux_wg (0: the same)
// for the further kinds of multi-kind modes.
hipError_t launch_finalize(const BatchHost& bh, int what, int kind, int gate, int producer_wg, double* hist,
                           int hist_stride, hipStream_t st, int aux_wg = 0);
hipError_t launch_update_r(const BatchHost& bh, int prec, int wg, hipStream_t st);
hipError_t launch_update_xd(const BatchHost& bh, int prec, int x_prec, int x_id, int wg, hipStream_t st);
hipError_t launch_copy_vec(const BatchHost& bh, int src_prec, int src_id, int dst_prec, int dst_id, int gate,
                           int wg, hipStream_t st);
hipError_t launch_add_lo_to_hi(const BatchHost& bh, int gate, int wg, hipStream_t st);  // x += x_lo ; x_lo = 0
hipError_t launch_zero_vec(const BatchHost& bh, int prec, int v_id, int gate, int wg, hipStream_t st);

// Finalize modes (one workgroup per slot, deterministic order).
enum Fin : int {
  FIN_B2 = 0,        // b2 = sum ; thr = tol^2 * b2 (tol from aux)
  FIN_START = 1,     // delta = sum ; state = (delta <= thr) ? 1 : 0 ; iter = 0
  FIN_ALPHA = 2,     // state 1 -> 2 ; else alpha = delta / dAd (breakdown -> NaN flag, state 2)
  FIN_BETA = 3,      // delta_old = delta ; delta = sum ; beta ; iter++ ; stop test
  FIN_TRUE = 4,      // aux = sqrt(sum / b2) (true residual)
  FIN_RELIABLE = 5,  // delta = sum (after the FP64 residual recomputation)
  FIN_ORTHO = 6,     // kinds 0,1,2 = Re<r,d>, Im<r,d>, |r|^2: c = 1 - <r,d>/|r|^2 ; delta = |r|^2
  FIN_FCG_ALPHA = 7, // kinds 0,1,2 = <d,Ad>, Re<d,r>, Im<d,r>: alpha = <d,r>/<d,Ad> (breakdown -> flag, state 2)
  FIN_FCG_RES = 8,   // kind 1 = |r|^2: delta, iter++, stop test
  FIN_FCG_BETA = 9   // kinds 1,2 = Re<Ad,z>, Im<Ad,z>: beta = -<Ad,z>/<d,Ad>
};
// Flexible CG vector stages (FP64; z, d, r, Ad, x are the V_Z, V_D, V_R, V_AD, V_X roles).
hipError_t launch_fcg_dir(const BatchHost& bh, int gate, int wg, hipStream_t st);      // d = z + beta d ; <d,r>
hipError_t launch_fcg_update(const BatchHost& bh, int wg, hipStream_t st);            // x += a d ; r -= a Ad ; |r|^2
hipError_t launch_fcg_beta_dot(const BatchHost& bh, int gate, int wg, hipStream_t st); // <Ad, z>
// Mixed precision, after a reliable update: restore <d, r> = |r|^2 for the new residual r.
hipError_t launch_rd_dot(const BatchHost& bh, int prec, int gate, int wg, hipStream_t st);
hipError_t launch_d_fix(const BatchHost& bh, int prec, int gate, int wg, hipStream_t st);

// Packing and conversions.  launch_pack_links packs FP64 (with lscale non-NULL it also writes the FP16
// scales) or FP32; FP16 comes from the packed FP64 matrices.
hipError_t launch_pack_links(int prec, const void* fat, const void* lng, double naik, const Geo& g, int antiper,
                             int par, void* out, float* lscale, hipStream_t st);
// FP16 packing from the FP64 packed matrices and the scales the FP64 pack wrote into lscale.
hipError_t launch_pack_f16_from_f64(const void* packed64, const float* lscale, const Geo& g, void* out,
                                    hipStream_t st);
hipError_t launch_convert_from_f64(int prec, const void* in, void* out, long nsites, hipStream_t st);
hipError_t launch_convert_to_f64(int prec, const void* in, void* out, long nsites, hipStream_t st);

Geo make_geo(const int dims[4]);

// Read-only streaming probe (probe.hip): bytes must be a positive multiple of stream_read_chunk_bytes();
// sink receives one word per chunk.
long stream_read_chunk_bytes();
hipError_t launch_stream_read(const void* buf, long bytes, unsigned* sink, hipStream_t st);

}  // namespace stag
