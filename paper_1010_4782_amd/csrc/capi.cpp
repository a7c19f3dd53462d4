// extern "C" entry points of libstagcg.so (declared in include/stagcg.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "fatten.h"
#include "noalloc.h"
#include "runtime.h"

namespace stag {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

hipError_t DevBuf::ensure(size_t need) {
  if (need <= bytes && ptr) return hipSuccess;
  release();
  if (need == 0) return hipSuccess;
  hipError_t e = hipMalloc(&ptr, need);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    return e;
  }
  bytes = need;
  return hipSuccess;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

hipError_t HostBuf::ensure(size_t need) {
  if (need <= bytes && ptr) return hipSuccess;
  release();
  if (need == 0) return hipSuccess;
  hipError_t e = hipHostMalloc(&ptr, need, hipHostMallocDefault);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    return e;
  }
  bytes = need;
  return hipSuccess;
}

void HostBuf::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

void Ctl::release() {
  for (int i = 0; i < kRing; ++i)
    if (ring_ev[i]) {
      (void)hipEventSynchronize(ring_ev[i]);
      (void)hipEventDestroy(ring_ev[i]);
      ring_ev[i] = nullptr;
    }
  probs.release();
  scal.release();
  partial.release();
  hist.release();
  h_scal.release();
  h_probs.release();
  ring_dev.release();
  ring_host.release();
}

ProbDev prob_dev(const stag_lattice_s* lat, int nrhs, int slot0) {
  ProbDev pd{};
  pd.g = lat->g;
  for (int p = 0; p < 3; ++p)
    for (int par = 0; par < 2; ++par) pd.links[p][par] = lat->links[p][par].ptr;
  for (int par = 0; par < 2; ++par) pd.lscale[par] = reinterpret_cast<const float*>(lat->lscale[par].ptr);
  pd.nrhs = nrhs;
  pd.slot0 = slot0;
  return pd;
}

}  // namespace stag

using namespace stag;

stag_lattice_s::~stag_lattice_s() {
  (void)hipDeviceSynchronize();
  for (auto& a : links)
    for (auto& b : a) b.release();
  for (auto& b : lscale) b.release();
  for (auto& b : vec) b.release();
  for (auto& b : io_lo) b.release();
  fat_ws.release();
  ctl.release();
  for (auto ev : prof_events) (void)hipEventDestroy(ev);
}

#define STAG_GUARD_BEGIN try {
#define STAG_GUARD_END                                   \
  }                                                      \
  catch (const std::bad_alloc&) {                        \
    set_error("host allocation failed");                 \
    return STAG_ERR_NOMEM;                               \
  }                                                      \
  catch (const std::exception& ex) {                     \
    set_error(std::string("internal error: ") + ex.what()); \
    return STAG_ERR_STATE;                               \
  }

namespace {

stag_status arg_error(const char* m) {
  set_error(m);
  return STAG_ERR_ARG;
}

// A parameter block in device memory for an asynchronous call, staged through
// pinned host memory.  Entries are reused round-robin once their event has passed.
struct RingEntry {
  char* host;
  char* dev;
  int idx;
};

stag_status ring_acquire(Ctl& c, size_t need, RingEntry& out) {
  need = (need + 255) & ~size_t(255);
  if (need > c.ring_entry) {
    for (int i = 0; i < Ctl::kRing; ++i)
      if (c.ring_used[i]) STAG_HIP_TRY(hipEventSynchronize(c.ring_ev[i]));
    c.ring_dev.release();
    c.ring_host.release();
    c.ring_entry = std::max(need, size_t(8192));
    STAG_HIP_TRY(c.ring_dev.ensure(c.ring_entry * Ctl::kRing));
    STAG_HIP_TRY(c.ring_host.ensure(c.ring_entry * Ctl::kRing));
    for (int i = 0; i < Ctl::kRing; ++i) c.ring_used[i] = false;
  }
  const int i = c.ring_next;
  c.ring_next = (i + 1) % Ctl::kRing;
  if (!c.ring_ev[i]) STAG_HIP_TRY(hipEventCreateWithFlags(&c.ring_ev[i], hipEventDisableTiming));
  if (c.ring_used[i]) STAG_HIP_TRY(hipEventSynchronize(c.ring_ev[i]));
  out.host = reinterpret_cast<char*>(c.ring_host.ptr) + i * c.ring_entry;
  out.dev = reinterpret_cast<char*>(c.ring_dev.ptr) + i * c.ring_entry;
  out.idx = i;
  return STAG_OK;
}

stag_status ring_release(Ctl& c, const RingEntry& e, hipStream_t st) {
  STAG_HIP_TRY(hipEventRecord(c.ring_ev[e.idx], st));
  c.ring_used[e.idx] = true;
  return STAG_OK;
}

// Set up a single-problem batch whose table, scalars and partials live in a ring entry.
stag_status single_batch(stag_lattice_s* L, int nrhs, const double* mass, void* const* vec_override, hipStream_t st,
                         BatchHost& bh, RingEntry& e, const Geo* geo_override = nullptr) {
  const int pstride = ceil_div(L->g.half, kWave / 2);  // 32-site partials of the time-streaming kernel
  const size_t off_scal = (sizeof(ProbDev) + 255) & ~size_t(255);
  const size_t off_part = off_scal + ((sizeof(Scal) * nrhs + 255) & ~size_t(255));
  const size_t need = off_part + sizeof(double) * (size_t)nrhs * kPartialSlots * pstride;
  stag_status s = ring_acquire(L->ctl, need, e);
  if (s != STAG_OK) return s;
  ProbDev pd = prob_dev(L, nrhs, 0);
  if (geo_override) pd.g = *geo_override;
  for (int v = 0; v < kNumVec; ++v) pd.vec[v] = L->vec[v].ptr;
  for (int v = 0; v < kNumVec; ++v)
    if (vec_override[v]) pd.vec[v] = vec_override[v];
  std::memcpy(e.host, &pd, sizeof(pd));
  Scal* sc = reinterpret_cast<Scal*>(e.host + off_scal);
  for (int r = 0; r < nrhs; ++r) {
    Scal z{};
    z.mass4 = mass ? 4.0 * mass[r] * mass[r] : 0.0;
    sc[r] = z;
  }
  STAG_HIP_TRY(hipMemcpyAsync(e.dev, e.host, off_part, hipMemcpyHostToDevice, st));
  bh.probs.assign(1, HostProb{pd.g.half, nrhs, 0, pd.g.Xh, pd.g.L[1], pd.g.L[2], pd.g.L[3], pd.g.t_open});
  bh.d_probs = reinterpret_cast<const ProbDev*>(e.dev);
  bh.d_scal = reinterpret_cast<Scal*>(e.dev + off_scal);
  bh.d_partial = reinterpret_cast<double*>(e.dev + off_part);
  bh.pstride = pstride;
  bh.nslots = nrhs;
  bh.max_half = pd.g.half;
  bh.long12 = L->g.long12 != 0;
  return STAG_OK;
}

std::string single_key(const BatchHost& bh, const stag_lattice_s* L, int prec) {
  std::vector<const stag_lattice_s*> lats{L};
  return tune_key(bh, lats, prec);
}

stag_status check_lattice(stag_lattice_t lat) {
  if (!lat) return arg_error("lattice is NULL");
  if (!lat->loaded) {
    set_error("load_links has not been called on this lattice");
    return STAG_ERR_STATE;
  }
  int dev = -1;
  STAG_HIP_TRY(hipGetDevice(&dev));
  if (dev != lat->device) return arg_error("the current HIP device is not the lattice's device");
  return STAG_OK;
}

}  // namespace

extern "C" {

void stag_cg_params_default(stag_cg_params* prm) {
  if (!prm) return;
  std::memset(prm, 0, sizeof(*prm));
  prm->tol = 1e-10;
  prm->max_iter = 0;
  prm->prec = STAG_F64;
  prm->reliable_interval = 50;
  prm->reliable_delta = 0.1;
  prm->check_interval = 16;
  prm->max_restarts = 5;
  prm->precond = STAG_PRECOND_NONE;
  prm->net = nullptr;
  prm->stall_window = 10;
  prm->stall_ratio = 0.9;
  prm->profile = 0;
  prm->history_len = 0;
  prm->history = nullptr;
  prm->autotune = 0;
}

const char* stag_last_error(void) { return g_last_error.c_str(); }

stag_status stag_create_lattice(const int32_t dims[4], int32_t t_antiperiodic, stag_lattice_t* out) {
  STAG_GUARD_BEGIN
  if (!dims || !out) return arg_error("dims and out must not be NULL");
  *out = nullptr;
  long vol = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2 || dims[i] % 2) return arg_error("every extent must be even and >= 2");
    vol *= dims[i];
    if (vol >= (1L << 31)) return arg_error("lattice volume must be below 2^31 sites");
  }
  if (t_antiperiodic != 0 && t_antiperiodic != 1) return arg_error("t_antiperiodic must be 0 or 1");
  int dev = 0;
  STAG_HIP_TRY(hipGetDevice(&dev));
  auto* L = new stag_lattice_s();
  for (int i = 0; i < 4; ++i) L->dims[i] = dims[i];
  L->antiper = t_antiperiodic;
  L->device = dev;
  L->g = make_geo(L->dims);
  L->g.antiper = t_antiperiodic;
  // the fixed workspace of stag_apply_m_noalloc: its address on this device, looked up once
  hipError_t he = noalloc_init(dev);
  if (he != hipSuccess) {
    delete L;
    set_error(std::string("HIP error: ") + hipGetErrorString(he));
    return STAG_ERR_HIP;
  }
  *out = L;
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_destroy_lattice(stag_lattice_t lat) {
  STAG_GUARD_BEGIN
  if (!lat) return arg_error("lattice is NULL");
  delete lat;
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_lattice_info(stag_lattice_t lat, int32_t dims[4], int64_t* half_volume) {
  if (!lat) return arg_error("lattice is NULL");
  if (dims)
    for (int i = 0; i < 4; ++i) dims[i] = lat->dims[i];
  if (half_volume) *half_volume = lat->g.half;
  return STAG_OK;
}

stag_status stag_load_links(stag_lattice_t lat, const void* fat, const void* lng, double naik_coeff,
                            uint32_t prec_mask, void* stream) {
  STAG_GUARD_BEGIN
  if (!lat) return arg_error("lattice is NULL");
  if (!fat) return arg_error("fat links must not be NULL");
  if (!std::isfinite(naik_coeff)) return arg_error("naik_coeff must be finite");
  if (prec_mask & ~(0x7u | STAG_LONG_SU3)) return arg_error("prec_mask has unknown bits");
  const bool c12 = (prec_mask & STAG_LONG_SU3) != 0;
  if (c12 && (!lng || naik_coeff == 0.0)) return arg_error("STAG_LONG_SU3 needs long links and a nonzero naik_coeff");
  int dev = -1;
  STAG_HIP_TRY(hipGetDevice(&dev));
  if (dev != lat->device) return arg_error("the current HIP device is not the lattice's device");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  prec_mask = (prec_mask & 0x7u) | STAG_PREC_BIT(STAG_F64);
  const size_t padded = (size_t)ceil_div(lat->g.half, kWave) * kWave;
  lat->loaded = false;
  lat->g.long12 = c12 ? 1 : 0;
  lat->g.cn_inv = c12 ? 1.0 / naik_coeff : 0.0;
  // FP64 is always packed; with FP16 requested too, the FP64 pack also computes the FP16 scales and the
  // FP16 matrices are converted from the packed FP64 ones
  const bool f16 = (prec_mask & STAG_PREC_BIT(P16)) != 0;
  for (int p = 0; p < 3; ++p) {
    if (!(prec_mask & STAG_PREC_BIT(p))) {
      for (auto& b : lat->links[p]) b.release();
      continue;
    }
    for (int par = 0; par < 2; ++par) {
      STAG_HIP_TRY(lat->links[p][par].ensure(padded / kWave * link_block_bytes(p, c12)));
      float* ls = nullptr;
      if (p == P16 || (p == P64 && f16)) {
        STAG_HIP_TRY(lat->lscale[par].ensure(padded * 2 * sizeof(float)));
        ls = reinterpret_cast<float*>(lat->lscale[par].ptr);
      }
      if (p == P16)
        STAG_HIP_TRY(launch_pack_f16_from_f64(lat->links[P64][par].ptr, ls, lat->g, lat->links[p][par].ptr, st));
      else
        STAG_HIP_TRY(launch_pack_links(p, fat, lng, naik_coeff, lat->g, lat->antiper, par, lat->links[p][par].ptr, ls,
                                       st));
    }
  }
  lat->built = prec_mask;
  lat->has_long = lng != nullptr;
  lat->naik = naik_coeff;
  lat->loaded = true;
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_dslash(stag_lattice_t lat, int32_t out_parity, const void* in, void* out, int32_t nrhs, int32_t prec,
                        void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (out_parity != 0 && out_parity != 1) return arg_error("out_parity must be 0 or 1");
  if (!in || !out) return arg_error("in and out must not be NULL");
  if (in == out) return arg_error("in and out must not overlap");
  if (nrhs < 1) return arg_error("nrhs must be >= 1");
  if (prec < STAG_F64 || prec > STAG_F16) return arg_error("prec must be STAG_F64, STAG_F32 or STAG_F16");
  if (!(lat->built & STAG_PREC_BIT(prec))) return arg_error("the requested precision was not packed by load_links");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* ov[kNumVec] = {};
  const long nsites = (long)lat->g.half * nrhs;
  if (prec == STAG_F64) {
    ov[V_D] = const_cast<void*>(in);
    ov[V_T] = out;
  } else {
    STAG_HIP_TRY(lat->io_lo[0].ensure(spinor_field_bytes(lat, prec, nrhs)));
    STAG_HIP_TRY(lat->io_lo[1].ensure(spinor_field_bytes(lat, prec, nrhs)));
    STAG_HIP_TRY(launch_convert_from_f64(prec, in, lat->io_lo[0].ptr, nsites, st));
    ov[V_D] = lat->io_lo[0].ptr;
    ov[V_T] = lat->io_lo[1].ptr;
  }
  BatchHost bh;
  RingEntry e;
  s = single_batch(lat, nrhs, nullptr, ov, st, bh, e);
  if (s != STAG_OK) return s;
  const DslashShape sh = lookup_shape(bh, single_key(bh, lat, prec), prec);
  STAG_HIP_TRY(launch_dslash(bh, prec, EPI_PLAIN, out_parity, V_D, V_T, 0, 0, 3, sh, st));
  if (prec != STAG_F64) STAG_HIP_TRY(launch_convert_to_f64(prec, lat->io_lo[1].ptr, out, nsites, st));
  return ring_release(lat->ctl, e, st);
  STAG_GUARD_END
}

stag_status stag_dslash_slab(stag_lattice_t lat, int32_t out_parity, int32_t t0, int32_t lt, const void* in_ext,
                             void* out, int32_t nrhs, int32_t prec, void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  const int Lt = lat->dims[3];
  if (out_parity != 0 && out_parity != 1) return arg_error("out_parity must be 0 or 1");
  if (t0 < 0 || t0 % 2 || lt < 2 || lt % 2 || t0 + lt > Lt)
    return arg_error("the slab [t0, t0 + lt) must lie in [0, Lt) with t0 and lt even, lt >= 2");
  if (!in_ext || !out) return arg_error("in_ext and out must not be NULL");
  if (nrhs < 1) return arg_error("nrhs must be >= 1");
  if (prec < STAG_F64 || prec > STAG_F16) return arg_error("prec must be STAG_F64, STAG_F32 or STAG_F16");
  if (!(lat->built & STAG_PREC_BIT(prec))) return arg_error("the requested precision was not packed by load_links");
  const long slice = lat->g.stride[3];  // sites of one parity in one time slice
  const long in_sites = slice * (lt + 6), out_sites = slice * lt;
  {
    const char* a = static_cast<const char*>(in_ext);
    const char* b = static_cast<const char*>(out);
    if (a < b + (size_t)out_sites * 48 * nrhs && b < a + (size_t)in_sites * 48 * nrhs)
      return arg_error("in_ext and out must not overlap");
  }
  Geo gs = lat->g;
  gs.L[3] = lt;
  gs.half = (int)out_sites;
  gs.in_half = (int)in_sites;
  gs.h1[3] = 1;
  gs.h3[3] = 3;
  gs.t0 = t0;
  gs.t_open = 1;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* ov[kNumVec] = {};
  const size_t vb = spinor_bytes(prec);
  if (prec == STAG_F64) {
    ov[V_D] = const_cast<char*>(static_cast<const char*>(in_ext)) + 3 * slice * vb;  // first interior slice
    ov[V_T] = out;
  } else {
    STAG_HIP_TRY(lat->io_lo[0].ensure(vb * in_sites * nrhs));
    STAG_HIP_TRY(lat->io_lo[1].ensure(vb * out_sites * nrhs));
    STAG_HIP_TRY(launch_convert_from_f64(prec, in_ext, lat->io_lo[0].ptr, in_sites * nrhs, st));
    ov[V_D] = static_cast<char*>(lat->io_lo[0].ptr) + 3 * slice * vb;
    ov[V_T] = lat->io_lo[1].ptr;
  }
  BatchHost bh;
  RingEntry e;
  s = single_batch(lat, nrhs, nullptr, ov, st, bh, e, &gs);
  if (s != STAG_OK) return s;
  const DslashShape sh = lookup_shape(bh, single_key(bh, lat, prec), prec);
  STAG_HIP_TRY(launch_dslash(bh, prec, EPI_PLAIN, out_parity, V_D, V_T, 0, 0, 3, sh, st));
  if (prec != STAG_F64) STAG_HIP_TRY(launch_convert_to_f64(prec, lat->io_lo[1].ptr, out, out_sites * nrhs, st));
  return ring_release(lat->ctl, e, st);
  STAG_GUARD_END
}

stag_status stag_apply_m(stag_lattice_t lat, const double* mass, const void* in, void* out, int32_t nrhs,
                         void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (!mass || !in || !out) return arg_error("mass, in and out must not be NULL");
  if (in == out) return arg_error("in and out must not overlap");
  if (nrhs < 1) return arg_error("nrhs must be >= 1");
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(mass[r])) return arg_error("mass must be finite");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  STAG_HIP_TRY(lat->vec[V_TMPO].ensure(spinor_field_bytes(lat, P64, nrhs)));
  void* ov[kNumVec] = {};
  ov[V_D] = const_cast<void*>(in);
  ov[V_AD] = out;
  BatchHost bh;
  RingEntry e;
  s = single_batch(lat, nrhs, mass, ov, st, bh, e);
  if (s != STAG_OK) return s;
  const DslashShape sh = lookup_shape(bh, single_key(bh, lat, P64), P64);
  STAG_HIP_TRY(launch_dslash(bh, P64, EPI_PLAIN, 1, V_D, V_TMPO, 0, 0, 3, sh, st));
  STAG_HIP_TRY(launch_dslash(bh, P64, EPI_XPAY, 0, V_TMPO, V_AD, V_D, 0, 3, sh, st));
  return ring_release(lat->ctl, e, st);
  STAG_GUARD_END
}

stag_status stag_fatten_links(stag_lattice_t lat, const void* thin, double u0, void* fat, void* lng,
                              void* stream) {
  STAG_GUARD_BEGIN
  if (!lat) return arg_error("lattice is NULL");
  if (!thin || !fat || !lng) return arg_error("thin, fat and lng must not be NULL");
  if (!std::isfinite(u0) || u0 <= 0.0) return arg_error("u0 must be finite and > 0");
  int dev = -1;
  STAG_HIP_TRY(hipGetDevice(&dev));
  if (dev != lat->device) return arg_error("the current HIP device is not the lattice's device");
  const size_t field = (size_t)4 * lat->g.half * 2 * 9 * 16;  // [4][V] 3x3 complex128
  auto overlap = [field](const void* a, const void* b) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + field && y < x + field;
  };
  if (overlap(thin, fat) || overlap(thin, lng) || overlap(fat, lng))
    return arg_error("thin, fat and lng must not overlap");
  STAG_HIP_TRY(lat->fat_ws.ensure(fatten_workspace_bytes(lat->dims)));
  STAG_HIP_TRY(fatten_links(lat->dims, thin, u0, fat, lng, lat->fat_ws.ptr, reinterpret_cast<hipStream_t>(stream)));
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_apply_m_noalloc(stag_lattice_t lat, const double* mass, const void* in, void* out, int32_t nrhs,
                                 void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (!mass || !in || !out) return arg_error("mass, in and out must not be NULL");
  if (in == out) return arg_error("in and out must not overlap");
  if (nrhs < 1 || nrhs > kNoAllocMaxRhs) return arg_error("stag_apply_m_noalloc: nrhs must be in [1, 64]");
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(mass[r])) return arg_error("mass must be finite");
  const size_t tmp = spinor_field_bytes(lat, P64, nrhs);
  if (tmp > kNoAllocBytes - kNoAllocParamBytes)
    return arg_error("stag_apply_m_noalloc: nrhs x V/2 x 48 bytes exceeds the fixed workspace (64 MiB - 16 KiB)");
  unsigned char* base = nullptr;
  STAG_HIP_TRY(noalloc_address(lat->device, &base));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ProbDev pd = prob_dev(lat, nrhs, 0);
  pd.vec[V_D] = const_cast<void*>(in);
  pd.vec[V_AD] = out;
  pd.vec[V_TMPO] = base + kNoAllocParamBytes;
  STAG_HIP_TRY(noalloc_write_params(base, pd, mass, nrhs, st));
  BatchHost bh;
  bh.probs.assign(1, HostProb{pd.g.half, nrhs, 0, pd.g.Xh, pd.g.L[1], pd.g.L[2], pd.g.L[3], pd.g.t_open});
  bh.d_probs = reinterpret_cast<const ProbDev*>(base);
  bh.d_scal = reinterpret_cast<Scal*>(base + noalloc_scal_offset());
  bh.d_partial = nullptr;  // the plain and xpay epilogues write no partial sums
  bh.pstride = 0;
  bh.nslots = nrhs;
  bh.max_half = pd.g.half;
  bh.long12 = lat->g.long12 != 0;
  const DslashShape sh = lookup_shape(bh, single_key(bh, lat, P64), P64);
  STAG_HIP_TRY(launch_dslash(bh, P64, EPI_PLAIN, 1, V_D, V_TMPO, 0, 0, 3, sh, st));
  STAG_HIP_TRY(launch_dslash(bh, P64, EPI_XPAY, 0, V_TMPO, V_AD, V_D, 0, 3, sh, st));
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_slice_norm2(stag_lattice_t lat, const void* v, int32_t nrhs, int32_t group, double weight,
                             int32_t accumulate, double* out, void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (!v || !out) return arg_error("v and out must not be NULL");
  if (nrhs < 1 || group < 1 || nrhs % group) return arg_error("group must be >= 1 and divide nrhs >= 1");
  if (!std::isfinite(weight)) return arg_error("weight must be finite");
  if (accumulate != 0 && accumulate != 1) return arg_error("accumulate must be 0 or 1");
  const int lt = lat->dims[3];
  STAG_HIP_TRY(launch_slice_norm2(v, lat->g.half, lat->g.half / lt, lt, nrhs / group, group, weight, accumulate, out,
                                  reinterpret_cast<hipStream_t>(stream)));
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_pion_correlator(stag_lattice_t lat, const void* chi, int32_t nsrc, double mass, double* out,
                                 void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (!chi || !out) return arg_error("chi and out must not be NULL");
  if (nsrc < 1) return arg_error("nsrc must be >= 1");
  if (!std::isfinite(mass)) return arg_error("mass must be finite");
  const int nrhs = 3 * nsrc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  STAG_HIP_TRY(lat->vec[V_TMPO].ensure(spinor_field_bytes(lat, P64, nrhs)));
  void* ov[kNumVec] = {};
  ov[V_D] = const_cast<void*>(chi);
  BatchHost bh;
  RingEntry e;
  s = single_batch(lat, nrhs, nullptr, ov, st, bh, e);
  if (s != STAG_OK) return s;
  const DslashShape sh = lookup_shape(bh, single_key(bh, lat, P64), P64);
  STAG_HIP_TRY(launch_dslash(bh, P64, EPI_PLAIN, 1, V_D, V_TMPO, 0, 0, 3, sh, st));
  s = ring_release(lat->ctl, e, st);
  if (s != STAG_OK) return s;
  const int lt = lat->dims[3];
  const long half = lat->g.half;
  // |D_oe chi|^2 = |G_o|^2 (the sign of G_o does not enter); the even part carries (2m)^2
  STAG_HIP_TRY(launch_slice_norm2(chi, half, half / lt, lt, nsrc, 3, 4.0 * mass * mass, 0, out, st));
  STAG_HIP_TRY(launch_slice_norm2(lat->vec[V_TMPO].ptr, half, half / lt, lt, nsrc, 3, 1.0, 1, out, st));
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_cg_solve(stag_lattice_t lat, const double* mass, const void* b, void* x, int32_t nrhs,
                          const stag_cg_params* prm, stag_cg_info* info, void* stream) {
  STAG_GUARD_BEGIN
  if (!lat) return arg_error("lattice is NULL");
  stag_problem p{lat, nrhs, mass, b, x};
  return solve_batch(1, &p, prm, info, reinterpret_cast<hipStream_t>(stream));
  STAG_GUARD_END
}

stag_status stag_cg_solve_batch(int32_t nprob, const stag_problem* probs, const stag_cg_params* prm,
                                stag_cg_info* info, void* stream) {
  STAG_GUARD_BEGIN
  return solve_batch(nprob, probs, prm, info, reinterpret_cast<hipStream_t>(stream));
  STAG_GUARD_END
}

stag_status stag_tune_dslash(stag_lattice_t lat, int32_t prec, int32_t nrhs, stag_shape* best, stag_shape* all,
                             int32_t max_all, int32_t* n_all, void* stream) {
  STAG_GUARD_BEGIN
  stag_status s = check_lattice(lat);
  if (s != STAG_OK) return s;
  if (nrhs < 1) return arg_error("nrhs must be >= 1");
  if (prec < STAG_F64 || prec > STAG_F16) return arg_error("prec must be STAG_F64, STAG_F32 or STAG_F16");
  if (!(lat->built & STAG_PREC_BIT(prec))) return arg_error("the requested precision was not packed by load_links");
  if (all && max_all < 0) return arg_error("max_all must be >= 0");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  STAG_HIP_TRY(lat->vec[V_D].ensure(spinor_field_bytes(lat, prec, nrhs)));
  STAG_HIP_TRY(lat->vec[V_T].ensure(spinor_field_bytes(lat, prec, nrhs)));
  STAG_HIP_TRY(hipMemsetAsync(lat->vec[V_D].ptr, 0, spinor_field_bytes(lat, prec, nrhs), st));
  void* ov[kNumVec] = {};
  BatchHost bh;
  RingEntry e;
  s = single_batch(lat, nrhs, nullptr, ov, st, bh, e);
  if (s != STAG_OK) return s;
  DslashShape b{};
  std::vector<std::pair<DslashShape, float>> timed;
  STAG_HIP_TRY(tune_batch(bh, single_key(bh, lat, prec), prec, st, &b, &timed));
  s = ring_release(lat->ctl, e, st);
  if (s != STAG_OK) return s;
  float best_us = 0.f;
  for (const auto& t : timed)
    if (t.first.wg == b.wg && t.first.r == b.r && t.first.lds == b.lds && t.first.order == b.order &&
        t.first.chunks == b.chunks)
      best_us = t.second;
  if (best) *best = stag_shape{b.wg, b.r, b.lds, b.order, b.chunks, best_us};
  if (all) {
    int n = 0;
    for (const auto& t : timed) {
      if (n >= max_all) break;
      all[n++] = stag_shape{t.first.wg, t.first.r, t.first.lds, t.first.order, t.first.chunks, t.second};
    }
    if (n_all) *n_all = n;
  }
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_set_dslash_shape(stag_lattice_t lat, int32_t prec, int32_t nrhs, const stag_shape* shape) {
  STAG_GUARD_BEGIN
  if (!lat) return arg_error("lattice is NULL");
  if (nrhs < 1) return arg_error("nrhs must be >= 1");
  if (prec < STAG_F64 || prec > STAG_F16) return arg_error("prec must be STAG_F64, STAG_F32 or STAG_F16");
  BatchHost bh;
  bh.probs.assign(1, HostProb{lat->g.half, nrhs, 0, lat->g.Xh, lat->g.L[1], lat->g.L[2], lat->g.L[3], 0});
  bh.long12 = lat->g.long12 != 0;
  const std::string key = single_key(bh, lat, prec);
  if (!shape || shape->wg == 0) {
    pin_shape(key, DslashShape{0, 1, 0, 0, 1});
    return STAG_OK;
  }
  const int wg = shape->wg, r = shape->rhs_per_lane;
  if (wg != 64 && wg != 128 && wg != 256) return arg_error("wg must be 0, 64, 128 or 256");
  if (r != 1 && r != 2 && r != 4 && r != 8) return arg_error("rhs_per_lane must be 1, 2, 4 or 8");
  if (nrhs % r) return arg_error("rhs_per_lane must divide nrhs");
  if (shape->lds_stage != 0 && shape->lds_stage != 1) return arg_error("lds_stage must be 0 or 1");
  if (shape->tile_order < 0 || shape->tile_order > 2) return arg_error("tile_order must be 0, 1 or 2");
  const int chunks = shape->tile_order != 0 ? shape->t_chunks : 1;
  if (chunks < 1) return arg_error("t_chunks must be >= 1 with tile_order 1 or 2");
  const DslashShape sh{wg, r, shape->lds_stage, shape->tile_order, chunks};
  if (!dslash_shape_valid(bh, prec, sh))
    return arg_error(sh.order == 2 ? "tile_order 2 needs FP16, wg 64, rhs_per_lane 8 or 4, no LDS staging, nrhs "
                                     "divisible by 8, Lx Ly Lz / 2 divisible by the sites per wave (64 or 32) and Lt "
                                     "by 2 t_chunks"
                     : sh.order ? "tile_order 1 needs Lz divisible by 8 t_chunks and wg dividing Ly x Lx / 2 (and, "
                                  "staged, an LDS window within 64 KiB)"
                                : "the LDS window of this shape exceeds 64 KiB (use fewer sites or RHS per workgroup)");
  pin_shape(key, sh);
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_stream_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream) {
  STAG_GUARD_BEGIN
  if (!buf || !sink) return arg_error("buf and sink must not be NULL");
  if (bytes <= 0 || bytes % stream_read_chunk_bytes()) return arg_error("bytes must be a positive multiple of 32768");
  STAG_HIP_TRY(launch_stream_read(buf, (long)bytes, sink, reinterpret_cast<hipStream_t>(stream)));
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_tune_cache_save(const char* path) {
  STAG_GUARD_BEGIN
  if (!path) return arg_error("path is NULL");
  if (!save_table(path)) {
    set_error(std::string("cannot write ") + path);
    return STAG_ERR_ARG;
  }
  return STAG_OK;
  STAG_GUARD_END
}

stag_status stag_tune_cache_load(const char* path) {
  STAG_GUARD_BEGIN
  if (!path) return arg_error("path is NULL");
  int n = 0;
  if (!load_table(path, &n)) {
    set_error(std::string("cannot read a tuning table from ") + path);
    return STAG_ERR_ARG;
  }
  return STAG_OK;
  STAG_GUARD_END
}

}  // extern "C"

