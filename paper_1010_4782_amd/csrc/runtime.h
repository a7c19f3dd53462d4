// Host runtime of libstagcg: the lattice object, its device buffers and the solver entry points.
#pragma once

#include <string>
#include <vector>

#include "../../include/stagcg.h"
#include "launch.h"

namespace stag {

// Thread-local error message behind stag_last_error().
void set_error(const std::string& msg);

// A device buffer that grows on demand (old contents are not kept).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need);
  void release();
};

// Pinned host buffer that grows on demand.
struct HostBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need);
  void release();
};

// Launch shape of the Dslash for one (precision, nrhs, lattice) combination.

struct Lattice;

// Control buffers of a solve or of an asynchronous operator call.
struct Ctl {
  DevBuf probs, scal, partial, hist;
  HostBuf h_scal, h_probs;
  // ring of parameter blocks for asynchronous calls (stag_dslash / stag_apply_m)
  static constexpr int kRing = 16;
  DevBuf ring_dev;
  HostBuf ring_host;
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;
  size_t ring_entry = 0;
  void release();
};

}  // namespace stag

struct stag_lattice_s {
  int dims[4] = {0, 0, 0, 0};
  int antiper = 1;
  int device = 0;
  stag::Geo g{};
  bool loaded = false;
  bool has_long = false;
  double naik = 0.0;
  uint32_t built = 0;                 // STAG_PREC_BIT of packed precisions
  stag::DevBuf links[3][2];           // packed links per precision and output parity
  stag::DevBuf lscale[2];             // f16 link scales per output parity
  stag::DevBuf vec[stag::kNumVec];    // solver workspace per role (grown for the largest nrhs)
  stag::DevBuf io_lo[2];              // low-precision staging for stag_dslash (in, out)
  stag::DevBuf fat_ws;                // staple fields of stag_fatten_links
  stag::Ctl ctl;
  std::vector<hipEvent_t> prof_events;
  ~stag_lattice_s();
};

namespace stag {

// Fill the device-side description of a lattice (links of every built precision).
ProbDev prob_dev(const stag_lattice_s* lat, int nrhs, int slot0);

// Autotuner (autotune.cpp): launch shapes keyed by (precision, lattice shapes, right-hand sides).
std::string tune_key(const BatchHost& bh, const std::vector<const stag_lattice_s*>& lats, int prec);
DslashShape lookup_shape(const BatchHost& bh, const std::string& key, int prec);
void pin_shape(const std::string& key, const DslashShape& s);
bool has_shape(const std::string& key);
hipError_t tune_batch(const BatchHost& bh, const std::string& key, int prec, hipStream_t st, DslashShape* best,
                      std::vector<std::pair<DslashShape, float>>* all, int in_id = V_D, int out_id = V_T);
bool save_table(const char* path);
bool load_table(const char* path, int* n_loaded);

// Network (net.cpp).
stag_lattice_s* net_lattice(stag_net_s* n);
// STAG_OK if the network's lattice still holds FP32 links and its device is current.
stag_status net_check(stag_net_s* n);
hipError_t net_forward(stag_net_s* n, const void* in, void* out, hipStream_t st);

// Solvers (solver.cpp).
stag_status solve_batch(int nprob, const stag_problem* probs, const stag_cg_params* prm, stag_cg_info* info,
                        hipStream_t st);

inline size_t spinor_field_bytes(const stag_lattice_s* lat, int prec, int nrhs) {
  return (size_t)lat->g.half * spinor_bytes(prec) * (size_t)nrhs;
}

}  // namespace stag

#define STAG_HIP_TRY(expr)                                                                      \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) {                                                                     \
      stag::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                       \
      return _e == hipErrorOutOfMemory ? STAG_ERR_NOMEM : STAG_ERR_HIP;                         \
    }                                                                                           \
  } while (0)
