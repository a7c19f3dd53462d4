// CG drivers: plain FP64 CG (Fig. 1) and mixed-precision CG with reliable
// updates, over a batch of problems (one or more lattices, each with its own
// right-hand sides and masses).  Every stage is one launch over the whole
// batch; alpha, beta and the stopping state live on the device, and the host
// only polls the per-slot state every `check_interval` iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>

#include "runtime.h"

namespace stag {

namespace {

constexpr int kVecWG = 256;

struct Run {
  std::vector<stag_lattice_s*> lats;
  BatchHost bh;
  Ctl* ctl = nullptr;
  hipStream_t st = nullptr;
  int prec = P64;
  DslashShape shape;     // inner-iteration Dslash
  DslashShape shape64;   // FP64 Dslash of the true residual
  int hist_len = 0;
  int profile_every = 0;  // time the Dslash launches of every profile_every-th iteration (0: never)
  long iter_count = 0;
  std::vector<hipEvent_t>* events = nullptr;
  size_t ev_used = 0;
  Scal* h_scal = nullptr;
};

stag_status fail_arg(const std::string& m) {
  set_error(m);
  return STAG_ERR_ARG;
}

// STAG_DEBUG=1 in the environment prints the per-slot scalars at every host poll.
bool debug_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("STAG_DEBUG");
    return v && v[0] == '1';
  }();
  return on;
}

hipError_t pull_scal(Run& R, const char* where = "") {
  hipError_t e = hipMemcpyAsync(R.h_scal, R.bh.d_scal, sizeof(Scal) * R.bh.nslots, hipMemcpyDeviceToHost, R.st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(R.st);
  if (e == hipSuccess && debug_enabled())
    for (int s = 0; s < R.bh.nslots; ++s) {
      const Scal& c = R.h_scal[s];
      std::fprintf(stderr, "[stag] %-10s slot %d state %d iter %d flags %d delta %.6e dAd %.6e alpha %.6e beta %.6e aux %.6e\n",
                   where, s, c.state, c.iter, c.flags, c.delta, c.dAd, c.alpha, c.beta, c.aux);
    }
  return e;
}

hipError_t push_scal(Run& R) {
  hipError_t e = hipMemcpyAsync(R.bh.d_scal, R.h_scal, sizeof(Scal) * R.bh.nslots, hipMemcpyHostToDevice, R.st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(R.st);
}

// An event record costs a few microseconds of idle GPU (it waits for the preceding kernel and
// publishes a timestamp), so only sampled iterations are bracketed.
bool sample_iteration(Run& R) { return R.profile_every > 0 && (R.iter_count++ % R.profile_every) == 0; }

hipError_t record(Run& R, bool on) {
  if (!on) return hipSuccess;
  if (R.ev_used == R.events->size()) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    R.events->push_back(ev);
  }
  return hipEventRecord((*R.events)[R.ev_used++], R.st);
}

// V_R = b - M x (FP64), aux = ||V_R|| / ||b||, delta = |V_R|^2, for slots passing `gate`.
hipError_t true_residual(Run& R, int gate) {
  const DslashShape s64 = R.shape64;
  hipError_t e = launch_dslash(R.bh, P64, EPI_PLAIN, 1, V_X, V_TMPO, 0, 0, gate, s64, R.st);
  if (e == hipSuccess) e = launch_dslash(R.bh, P64, EPI_RESID, 0, V_TMPO, V_R, V_X, V_B, gate, s64, R.st);
  if (e == hipSuccess) e = launch_finalize(R.bh, FIN_TRUE, 1, gate, s64.wg, nullptr, 0, R.st);
  return e;
}

// One CG iteration in precision P (x accumulated in precision PX at x_id).
hipError_t iteration(Run& R, int x_prec, int x_id, double* d_hist) {
  const int P = R.prec;
  const bool samp = sample_iteration(R);
  hipError_t e = record(R, samp);
  if (e == hipSuccess) e = launch_dslash(R.bh, P, EPI_PLAIN, 1, V_D, V_T, 0, 0, 1, R.shape, R.st);
  if (e == hipSuccess) e = launch_dslash(R.bh, P, EPI_XPAY_DOT, 0, V_T, V_AD, V_D, 0, 1, R.shape, R.st);
  if (e == hipSuccess) e = record(R, samp);
  if (e == hipSuccess) e = launch_finalize(R.bh, FIN_ALPHA, 0, 2, partial_wg(R.shape), d_hist, R.hist_len, R.st);
  if (e == hipSuccess) e = launch_update_r(R.bh, P, kVecWG, R.st);
  if (e == hipSuccess) e = launch_finalize(R.bh, FIN_BETA, 1, 1, kVecWG, d_hist, R.hist_len, R.st);
  if (e == hipSuccess) e = launch_update_xd(R.bh, P, x_prec, x_id, kVecWG, R.st);
  return e;
}

// Flexible CG with the network preconditioner (FP64 vectors):
//   z = N(r); beta = -<A d_prev, z> / <d_prev, A d_prev>; d = z + beta d;
//   alpha = <d, r> / <d, A d>; x += alpha d; r -= alpha A d.
// The operator runs in the solve's precision: for FP32/FP16, d is rounded to that storage, A d is
// computed there (two Dslash launches, <d, A d> in the epilogue) and widened back to FP64, as in the
// mixed-precision CG.  Its rounding makes the iterated r drift from b - M x, so the host replaces r by
// the FP64 true residual ("reliable update") once the iterated |r| has dropped by reliable_delta since
// the last one, and before accepting an iterated convergence.  The direction d is kept (alpha is the
// exact line search along d for the new r, and the flexible recurrence needs no other relation
// between d and r); only <d, r> is recomputed.
// Every stall_window iterations (the first check after the first window) the host compares the
// smallest r^dag r of the window with the previous window's; a slot that did not drop below
// stall_ratio^2 times it (or broke down) leaves the phase, and the plain-CG passes that follow finish it
// from its current x.
stag_status fcg_phase(Run& R, const stag_cg_params& prm, const stag_problem& pb, double* d_hist, std::vector<int>& iters,
                      std::vector<int>& fell_back, std::vector<int>& n_rel) {
  const int nslots = R.bh.nslots;
  const int half = R.bh.probs[0].half;
  const size_t vb = (size_t)half * 48;
  const int P = R.prec;
  const bool lowp = P != P64;
  stag_lattice_s* L = pb.lat;
  char* rbase = reinterpret_cast<char*>(L->vec[V_R].ptr);
  char* zbase = reinterpret_cast<char*>(L->vec[V_Z].ptr);
  const int window = prm.stall_window > 0 ? prm.stall_window : 10;
  const double ratio2 = prm.stall_ratio * prm.stall_ratio;
  const double drop2 = (lowp && prm.reliable_delta > 0.0) ? prm.reliable_delta * prm.reliable_delta : 0.0;
  constexpr int kMaxFcgReliable = 64;  // reliable updates per slot before the phase gives the slot up
  STAG_HIP_TRY(pull_scal(R, "fcg-start"));
  std::vector<double> prev(nslots, 0.0);
  std::vector<char> part(nslots, 0);
  std::vector<char> active(nslots, 0);  // running at the last host poll: the network is applied to these
  std::vector<int> saved(nslots), nrel(nslots, 0);
  std::vector<char> done(nslots, 0);  // true residual below tol (after a reliable update)
  bool any = false;
  for (int s = 0; s < nslots; ++s) {
    Scal& sc = R.h_scal[s];
    saved[s] = sc.state;
    if (sc.state == 3 || sc.aux <= prm.tol) {  // zero source or already converged: not in the phase
      sc.state = 3;
      continue;
    }
    sc.state = 0;
    sc.iter = 0;
    sc.flags = 0;
    sc.br = sc.bi = 0.0;
    sc.dmin = sc.delta;
    sc.rel_thr = drop2 * sc.delta;
    prev[s] = sc.delta;
    part[s] = 1;
    active[s] = 1;
    any = true;
  }
  if (!any) {
    for (int s = 0; s < nslots; ++s) R.h_scal[s].state = saved[s];
    STAG_HIP_TRY(push_scal(R));
    return STAG_OK;
  }
  STAG_HIP_TRY(push_scal(R));
  auto apply_net = [&]() -> hipError_t {
    for (int r = 0; r < nslots; ++r) {
      if (!active[r]) continue;
      hipError_t e = net_forward(prm.net, rbase + r * vb, zbase + r * vb, R.st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // A d for the running slots, and <d, A d> in partial kind 0
  auto apply_a = [&]() -> hipError_t {
    if (!lowp) {
      hipError_t e = launch_dslash(R.bh, P64, EPI_PLAIN, 1, V_D, V_T, 0, 0, 1, R.shape64, R.st);
      if (e == hipSuccess) e = launch_dslash(R.bh, P64, EPI_XPAY_DOT, 0, V_T, V_AD, V_D, 0, 1, R.shape64, R.st);
      return e;
    }
    // d -> V_RL (storage precision), A d -> V_XL, widened into V_AD
    hipError_t e = launch_copy_vec(R.bh, P64, V_D, P, V_RL, 1, kVecWG, R.st);
    if (e == hipSuccess) e = launch_dslash(R.bh, P, EPI_PLAIN, 1, V_RL, V_T, 0, 0, 1, R.shape, R.st);
    if (e == hipSuccess) e = launch_dslash(R.bh, P, EPI_XPAY_DOT, 0, V_T, V_XL, V_RL, 0, 1, R.shape, R.st);
    if (e == hipSuccess) e = launch_copy_vec(R.bh, P, V_XL, P64, V_AD, 1, kVecWG, R.st);
    return e;
  };
  // the next direction of the running slots: z = N(r), beta, d = z + beta d and <d, r>
  auto next_dir = [&]() -> hipError_t {
    hipError_t e = apply_net();
    if (e == hipSuccess) e = launch_fcg_beta_dot(R.bh, 1, kVecWG, R.st);
    if (e == hipSuccess) e = launch_finalize(R.bh, FIN_FCG_BETA, 1, 1, kVecWG, nullptr, 0, R.st);
    if (e == hipSuccess) e = launch_fcg_dir(R.bh, 1, kVecWG, R.st);
    return e;
  };
  const int dot_wg = lowp ? partial_wg(R.shape) : R.shape64.wg;
  STAG_HIP_TRY(apply_net());
  STAG_HIP_TRY(launch_zero_vec(R.bh, P64, V_D, 1, kVecWG, R.st));
  STAG_HIP_TRY(launch_fcg_dir(R.bh, 1, kVecWG, R.st));  // d = z, <d, r>
  // A window ends after a residual update, before the network is applied to the new r: a slot that the
  // stall test hands over costs no network application it would not use, and a reliable update's true
  // residual is the one the network sees.
  for (;;) {
    for (int i = 0; i < window; ++i) {
      const bool samp = sample_iteration(R);
      hipError_t e = i > 0 ? next_dir() : hipSuccess;
      if (e == hipSuccess) e = record(R, samp);
      if (e == hipSuccess) e = apply_a();
      if (e == hipSuccess) e = record(R, samp);
      if (e == hipSuccess) e = launch_finalize(R.bh, FIN_FCG_ALPHA, 0, 1, dot_wg, d_hist, R.hist_len, R.st, kVecWG);
      if (e == hipSuccess) e = launch_fcg_update(R.bh, kVecWG, R.st);
      if (e == hipSuccess) e = launch_finalize(R.bh, FIN_FCG_RES, 1, 1, kVecWG, nullptr, 0, R.st);
      STAG_HIP_TRY(e);
    }
    STAG_HIP_TRY(pull_scal(R, "poll-fcg"));
    // stall test; slots due for a reliable update (iterated |r| dropped, or iterated convergence to check)
    std::vector<char> due(nslots, 0);
    bool any_due = false, running = false;
    for (int s = 0; s < nslots; ++s) {
      Scal& sc = R.h_scal[s];
      if (!part[s] || done[s]) continue;
      if (sc.state == 2) {  // broke down
        if (sc.flags & kFlagBreakdown) fell_back[s] = 1;
        continue;
      }
      if (sc.state == 1 && (sc.flags & kFlagMaxIter)) continue;
      // the residual of a preconditioned CG need not fall monotonically: compare the best r^dag r
      // of this window with the best one window earlier
      if (sc.state == 0 && sc.dmin > ratio2 * prev[s]) {
        fell_back[s] = 1;
        sc.state = 2;
        continue;
      }
      prev[s] = sc.dmin;
      const bool conv = sc.state == 1;  // iterated residual below the threshold
      if (lowp && (conv || sc.delta <= sc.rel_thr)) {
        if (nrel[s] >= kMaxFcgReliable) {
          sc.state = 1;
          continue;
        }
        due[s] = 1;
        any_due = true;
        sc.state = 1;  // the gate of the update kernels; running slots stay in state 0
      } else if (sc.state == 0) {
        running = true;
      }
    }
    STAG_HIP_TRY(push_scal(R));
    if (any_due) {
      // r = b - M x in FP64 for the slots in state 1, then <d, r> with the new r
      STAG_HIP_TRY(true_residual(R, 4));
      STAG_HIP_TRY(pull_scal(R, "fcg-reliable"));
      bool any_restart = false;
      for (int s = 0; s < nslots; ++s) {
        if (!due[s]) continue;
        Scal& sc = R.h_scal[s];
        nrel[s] += 1;
        if (sc.aux <= prm.tol) {
          sc.state = 3;  // converged; classified after the phase
          done[s] = 1;
          continue;
        }
        // continue from the true residual; the next window must bring r^dag r below stall_ratio^2 of it
        sc.rel_thr = drop2 * sc.delta;
        sc.dmin = sc.delta;
        prev[s] = sc.delta;
        any_restart = true;
      }
      if (any_restart)
        for (int s = 0; s < nslots; ++s)
          if (due[s] && !done[s]) {
            R.h_scal[s].state = 0;
            running = true;
          }
      for (int s = 0; s < nslots; ++s)
        if (done[s]) R.h_scal[s].state = 1;
      STAG_HIP_TRY(push_scal(R));
    }
    for (int s = 0; s < nslots; ++s) active[s] = part[s] && R.h_scal[s].state == 0;
    if (!running) break;
    STAG_HIP_TRY(next_dir());
  }
  // hand the participants back to the outer loop (state 2: classify) and restore the others
  for (int s = 0; s < nslots; ++s) {
    Scal& sc = R.h_scal[s];
    if (!part[s]) {
      sc.state = saved[s];
      continue;
    }
    iters[s] += sc.iter;
    n_rel[s] += nrel[s];
    sc.iter = 0;
    sc.flags &= ~(kFlagBreakdown | kFlagMaxIter);
    sc.state = 2;
  }
  STAG_HIP_TRY(push_scal(R));
  return STAG_OK;
}

}  // namespace

stag_status solve_batch(int nprob, const stag_problem* probs, const stag_cg_params* prm_in, stag_cg_info* info,
                        hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  stag_cg_params prm;
  if (prm_in) prm = *prm_in; else stag_cg_params_default(&prm);
  if (nprob < 1 || nprob > kMaxProb) return fail_arg("nprob must be in [1, 16]");
  if (!probs || !info) return fail_arg("probs and info must not be NULL");
  if (!(prm.tol > 0.0) || !std::isfinite(prm.tol)) return fail_arg("tol must be a positive finite number");
  if (prm.prec < STAG_F64 || prm.prec > STAG_F16) return fail_arg("prec must be STAG_F64, STAG_F32 or STAG_F16");
  if (prm.precond != STAG_PRECOND_NONE && prm.precond != STAG_PRECOND_NET) return fail_arg("unknown precond");
  const bool use_net = prm.precond == STAG_PRECOND_NET;
  if (use_net) {
    if (nprob != 1) return fail_arg("the network preconditioner solves one problem at a time");
    if (!prm.net) return fail_arg("precond = STAG_PRECOND_NET needs a network");
    if (net_lattice(prm.net) != probs[0].lat) return fail_arg("the network was built on another lattice");
    const stag_status c = net_check(prm.net);
    if (c != STAG_OK) return c;
    if (!(prm.stall_ratio > 0.0)) return fail_arg("stall_ratio must be positive");
  }
  if (prm.check_interval <= 0) prm.check_interval = 16;
  if (prm.reliable_interval <= 0) prm.reliable_interval = 50;
  if (prm.max_restarts < 0) prm.max_restarts = 0;
  if (prm.history_len < 0 || (prm.history_len > 0 && !prm.history)) return fail_arg("history_len > 0 needs a history buffer");

  Run R;
  R.st = st;
  R.prec = prm.prec;
  R.hist_len = prm.history_len;
  R.profile_every = std::max(0, prm.profile);
  std::set<stag_lattice_s*> seen;
  int nslots = 0, dev = -1;
  hipGetDevice(&dev);
  for (int p = 0; p < nprob; ++p) {
    const stag_problem& q = probs[p];
    if (!q.lat) return fail_arg("problem lattice is NULL");
    if (!q.lat->loaded) { set_error("load_links has not been called on a lattice of the batch"); return STAG_ERR_STATE; }
    if (q.nrhs < 1) return fail_arg("nrhs must be >= 1");
    if (!q.mass || !q.b || !q.x) return fail_arg("mass, b and x must not be NULL");
    {
      // x is rewritten while b is still read (true residual): the two may not overlap
      const char* b0 = static_cast<const char*>(q.b);
      const char* x0 = static_cast<const char*>(q.x);
      const size_t bytes = (size_t)q.lat->g.half * 48 * q.nrhs;
      if (b0 < x0 + bytes && x0 < b0 + bytes) return fail_arg("b and x must not overlap");
    }
    if (!(q.lat->built & STAG_PREC_BIT(prm.prec))) return fail_arg("the requested precision was not packed by load_links");
    if (q.lat->device != dev) return fail_arg("lattice belongs to another device than the current one");
    if (!seen.insert(q.lat).second) return fail_arg("a lattice may appear only once per batch (merge its right-hand sides)");
    if (q.lat->g.long12 != probs[0].lat->g.long12)
      return fail_arg("the lattices of a batch must all use the same long-link storage (STAG_LONG_SU3 or not)");
    for (int r = 0; r < q.nrhs; ++r)
      if (!std::isfinite(q.mass[r])) return fail_arg("mass must be finite");
    nslots += q.nrhs;
  }
  const bool mixed = prm.prec != STAG_F64;

  // ---- workspace and tables ----
  Ctl& ctl = probs[0].lat->ctl;
  R.ctl = &ctl;
  int max_half = 0;
  R.bh.probs.clear();
  std::vector<ProbDev> table(nprob);
  int slot = 0;
  for (int p = 0; p < nprob; ++p) {
    stag_lattice_s* L = probs[p].lat;
    const int n = probs[p].nrhs;
    R.lats.push_back(L);
    const int P = prm.prec;
    STAG_HIP_TRY(L->vec[V_R].ensure(spinor_field_bytes(L, P64, n)));
    STAG_HIP_TRY(L->vec[V_TMPO].ensure(spinor_field_bytes(L, P64, n)));
    STAG_HIP_TRY(L->vec[V_D].ensure(spinor_field_bytes(L, P, n)));
    STAG_HIP_TRY(L->vec[V_AD].ensure(spinor_field_bytes(L, P, n)));
    STAG_HIP_TRY(L->vec[V_T].ensure(spinor_field_bytes(L, P, n)));
    if (mixed) {
      STAG_HIP_TRY(L->vec[V_RL].ensure(spinor_field_bytes(L, P, n)));
      STAG_HIP_TRY(L->vec[V_XL].ensure(spinor_field_bytes(L, P32, n)));
    }
    if (use_net) {
      // flexible CG keeps d and Ad in FP64 whatever the inner precision of the plain-CG phase
      STAG_HIP_TRY(L->vec[V_Z].ensure(spinor_field_bytes(L, P64, n)));
      STAG_HIP_TRY(L->vec[V_D].ensure(spinor_field_bytes(L, P64, n)));
      STAG_HIP_TRY(L->vec[V_AD].ensure(spinor_field_bytes(L, P64, n)));
      STAG_HIP_TRY(L->vec[V_T].ensure(spinor_field_bytes(L, P64, n)));
    }
    ProbDev pd = prob_dev(L, n, slot);
    for (int v = 0; v < kNumVec; ++v) pd.vec[v] = L->vec[v].ptr;
    pd.vec[V_B] = const_cast<void*>(probs[p].b);
    pd.vec[V_X] = probs[p].x;
    table[p] = pd;
    R.bh.probs.push_back(HostProb{L->g.half, n, slot, L->g.Xh, L->g.L[1], L->g.L[2], L->g.L[3], 0});
    max_half = std::max(max_half, L->g.half);
    slot += n;
  }
  R.bh.nslots = nslots;
  R.bh.max_half = max_half;
  R.bh.long12 = probs[0].lat->g.long12 != 0;
  R.bh.pstride = ceil_div(max_half, kWave / 2);  // 32-site partials of the time-streaming kernel
  STAG_HIP_TRY(ctl.probs.ensure(sizeof(ProbDev) * kMaxProb));
  STAG_HIP_TRY(ctl.scal.ensure(sizeof(Scal) * nslots));
  STAG_HIP_TRY(ctl.partial.ensure(sizeof(double) * (size_t)nslots * kPartialSlots * R.bh.pstride));
  STAG_HIP_TRY(ctl.h_scal.ensure(sizeof(Scal) * nslots));
  STAG_HIP_TRY(ctl.h_probs.ensure(sizeof(ProbDev) * kMaxProb));
  double* d_hist = nullptr;
  if (R.hist_len > 0) {
    STAG_HIP_TRY(ctl.hist.ensure(sizeof(double) * 2 * (size_t)nslots * R.hist_len));
    d_hist = reinterpret_cast<double*>(ctl.hist.ptr);
    STAG_HIP_TRY(hipMemsetAsync(d_hist, 0, sizeof(double) * 2 * (size_t)nslots * R.hist_len, st));
  }
  R.bh.d_probs = reinterpret_cast<const ProbDev*>(ctl.probs.ptr);
  R.bh.d_scal = reinterpret_cast<Scal*>(ctl.scal.ptr);
  R.bh.d_partial = reinterpret_cast<double*>(ctl.partial.ptr);
  R.h_scal = reinterpret_cast<Scal*>(ctl.h_scal.ptr);
  R.events = &probs[0].lat->prof_events;
  std::memcpy(ctl.h_probs.ptr, table.data(), sizeof(ProbDev) * nprob);
  STAG_HIP_TRY(hipMemcpyAsync(ctl.probs.ptr, ctl.h_probs.ptr, sizeof(ProbDev) * nprob, hipMemcpyHostToDevice, st));
  {
    std::vector<const stag_lattice_s*> lats(R.lats.begin(), R.lats.end());
    const std::string key = tune_key(R.bh, lats, prm.prec);
    if (prm.autotune && !has_shape(key)) STAG_HIP_TRY(tune_batch(R.bh, key, prm.prec, st, nullptr, nullptr));
    R.shape = lookup_shape(R.bh, key, prm.prec);
    // the FP64 launches of the true residual use the FP64 key's shape; a mixed-precision solve tunes it on
    // the FP64 buffers those launches use (x, read only, into the residual scratch)
    const std::string key64 = tune_key(R.bh, lats, P64);
    if (prm.autotune && mixed && !has_shape(key64))
      STAG_HIP_TRY(tune_batch(R.bh, key64, P64, st, nullptr, nullptr, V_X, V_TMPO));
    R.shape64 = lookup_shape(R.bh, key64, P64);
  }

  // ---- scalars ----
  std::vector<int> passes(nslots, 0), iters(nslots, 0), n_rel(nslots, 0);
  slot = 0;
  for (int p = 0; p < nprob; ++p) {
    const int half = probs[p].lat->g.half;
    for (int r = 0; r < probs[p].nrhs; ++r, ++slot) {
      Scal s{};
      s.mass4 = 4.0 * probs[p].mass[r] * probs[p].mass[r];
      s.aux = prm.tol * prm.tol;
      s.max_iter = prm.max_iter > 0 ? prm.max_iter : 3 * half;
      s.hist_len = R.hist_len;
      s.state = 0;
      R.h_scal[slot] = s;
    }
  }
  STAG_HIP_TRY(push_scal(R));
  STAG_HIP_TRY(launch_norm2(R.bh, P64, V_B, 1, 3, kVecWG, st));
  STAG_HIP_TRY(launch_finalize(R.bh, FIN_B2, 1, 3, kVecWG, nullptr, 0, st));
  STAG_HIP_TRY(pull_scal(R));
  std::vector<char> zero_src(nslots, 0);
  bool any_zero = false;
  for (int s = 0; s < nslots; ++s) any_zero |= (zero_src[s] = R.h_scal[s].b2 == 0.0) != 0;
  if (any_zero) {
    // b = 0 has the solution x = 0: zero those x and leave the slots finished.
    for (int s = 0; s < nslots; ++s) R.h_scal[s].state = zero_src[s] ? 0 : 3;
    STAG_HIP_TRY(push_scal(R));
    STAG_HIP_TRY(launch_zero_vec(R.bh, P64, V_X, 1, kVecWG, st));
    for (int s = 0; s < nslots; ++s) {
      R.h_scal[s].state = zero_src[s] ? 3 : 0;
      if (zero_src[s]) R.h_scal[s].aux = 0.0;
    }
    STAG_HIP_TRY(push_scal(R));
  }

  // ---- restart loop: r = b - M x (FP64), decide, iterate ----
  STAG_HIP_TRY(true_residual(R, 0));
  std::vector<int> fell_back(nslots, 0);
  if (use_net) {
    stag_status fs = fcg_phase(R, prm, probs[0], d_hist, iters, fell_back, n_rel);
    if (fs != STAG_OK) return fs;
    STAG_HIP_TRY(true_residual(R, 0));
  }
  const int x_prec = mixed ? P32 : P64;
  const int x_id = mixed ? V_XL : V_X;
  std::vector<int> done_status(nslots, STAG_OK);
  for (;;) {
    STAG_HIP_TRY(pull_scal(R, "classify"));
    bool any_run = false;
    for (int s = 0; s < nslots; ++s) {
      Scal& sc = R.h_scal[s];
      if (sc.state == 3) continue;
      iters[s] += sc.iter;
      if (sc.aux <= prm.tol) {
        sc.state = 3;
        done_status[s] = STAG_OK;
      } else if ((sc.flags & kFlagNaN) || !std::isfinite(sc.aux)) {
        sc.state = 3;
        done_status[s] = STAG_ERR_NAN;
      } else if (passes[s] > prm.max_restarts) {
        sc.state = 3;
        done_status[s] = STAG_ERR_NOT_CONVERGED;
      } else {
        sc.state = 0;
        sc.iter = 0;
        sc.flags = 0;
        sc.rel_thr = (mixed && prm.reliable_delta > 0.0) ? prm.reliable_delta * prm.reliable_delta * sc.delta : 0.0;
        passes[s] += 1;
        any_run = true;
      }
    }
    STAG_HIP_TRY(push_scal(R));
    if (!any_run) break;
    if (!mixed) {
      STAG_HIP_TRY(launch_copy_vec(R.bh, P64, V_R, P64, V_D, 1, kVecWG, st));
      for (;;) {
        for (int i = 0; i < prm.check_interval; ++i) STAG_HIP_TRY(iteration(R, x_prec, x_id, d_hist));
        STAG_HIP_TRY(pull_scal(R));
        bool running = false;
        for (int s = 0; s < nslots; ++s) running |= R.h_scal[s].state == 0;
        if (!running) break;
      }
    } else {
      const int P = prm.prec;
      STAG_HIP_TRY(launch_copy_vec(R.bh, P64, V_R, P, V_RL, 1, kVecWG, st));
      STAG_HIP_TRY(launch_copy_vec(R.bh, P, V_RL, P, V_D, 1, kVecWG, st));
      STAG_HIP_TRY(launch_zero_vec(R.bh, P32, V_XL, 1, kVecWG, st));
      int since = 0;
      std::vector<char> parked(nslots, 0);
      const double drop2 = prm.reliable_delta > 0.0 ? prm.reliable_delta * prm.reliable_delta : 0.0;
      for (;;) {
        // a batch ends where the next interval-driven reliable update is due, so that it comes after
        // exactly reliable_interval iterations, not at the next multiple of check_interval
        const int batch = std::min(prm.check_interval, std::max(1, prm.reliable_interval - since));
        for (int i = 0; i < batch; ++i) STAG_HIP_TRY(iteration(R, x_prec, x_id, d_hist));
        since += batch;
        STAG_HIP_TRY(pull_scal(R, "poll-mp"));
        // Slots that stopped (apparent convergence, residual drop, iteration cap) wait for a
        // reliable update; once reliable_interval iterations have passed, every running slot does.
        bool any_wait = false, running = false;
        for (int s = 0; s < nslots; ++s) {
          Scal& sc = R.h_scal[s];
          if ((sc.state == 1 || sc.state == 2) && !(sc.flags & kFlagNaN)) {
            sc.state = 1;
            any_wait = true;
          }
          running |= sc.state == 0;
        }
        if (!running && !any_wait) {  // everything parked or broken down
          for (int s = 0; s < nslots; ++s)
            if (parked[s]) R.h_scal[s].state = 2;
          STAG_HIP_TRY(push_scal(R));
          break;
        }
        const bool interval_due = since >= prm.reliable_interval;
        if (!any_wait && !interval_due) continue;
        if (interval_due)
          for (int s = 0; s < nslots; ++s)
            if (R.h_scal[s].state == 0) R.h_scal[s].state = 1;
        // the interval restarts once every running slot is being updated (always, for one RHS)
        bool any_running = false;
        for (int s = 0; s < nslots; ++s) any_running |= R.h_scal[s].state == 0;
        if (!any_running) since = 0;
        STAG_HIP_TRY(push_scal(R));
        // reliable update (slots in state 1): x += x_lo, r = b - M x in FP64, r_lo = r, and
        // restore <d, r> = |r|^2 for the new residual.
        STAG_HIP_TRY(launch_add_lo_to_hi(R.bh, 4, kVecWG, st));
        STAG_HIP_TRY(true_residual(R, 4));
        STAG_HIP_TRY(launch_copy_vec(R.bh, P64, V_R, P, V_RL, 4, kVecWG, st));
        STAG_HIP_TRY(launch_rd_dot(R.bh, P, 4, kVecWG, st));
        STAG_HIP_TRY(launch_finalize(R.bh, FIN_ORTHO, 0, 4, kVecWG, nullptr, 0, st));
        STAG_HIP_TRY(launch_d_fix(R.bh, P, 4, kVecWG, st));
        STAG_HIP_TRY(pull_scal(R, "reliable"));
        bool cont = running;
        for (int s = 0; s < nslots; ++s) {
          Scal& sc = R.h_scal[s];
          if (sc.state != 1) continue;
          n_rel[s] += 1;
          sc.flags &= ~kFlagRelDue;
          if (sc.aux <= prm.tol || (sc.flags & kFlagMaxIter)) {
            sc.state = 3;  // out of the inner loop; the outer loop classifies it
            parked[s] = 1;
          } else {
            sc.state = 0;
            sc.rel_thr = drop2 * sc.delta;
            cont = true;
          }
        }
        if (!cont)
          for (int s = 0; s < nslots; ++s)
            if (parked[s]) R.h_scal[s].state = 2;
        STAG_HIP_TRY(push_scal(R));
        if (!cont) break;
      }
    }
    STAG_HIP_TRY(true_residual(R, 0));
  }

  // ---- results ----
  std::vector<double> hist;
  if (R.hist_len > 0) {
    hist.resize(2 * (size_t)nslots * R.hist_len);
    STAG_HIP_TRY(hipMemcpyAsync(hist.data(), d_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  STAG_HIP_TRY(hipStreamSynchronize(st));
  if (R.hist_len > 0) std::memcpy(prm.history, hist.data(), hist.size() * sizeof(double));
  // A sampled iteration brackets its two back-to-back Dslash launches with one pair of events
  // (an event between them would add its own idle time to both).  Iterations whose slots had
  // all stopped return at once (a few us); only pairs that did work (at least a quarter of the
  // median) enter the Dslash timing.
  double dms = 0.0;
  int dcalls = 0;
  if (R.profile_every > 0) {
    std::vector<float> dur;
    for (size_t i = 0; i + 1 < R.ev_used; i += 2) {
      float a = 0.f;
      STAG_HIP_TRY(hipEventElapsedTime(&a, (*R.events)[i], (*R.events)[i + 1]));
      dur.push_back(a);
    }
    if (!dur.empty()) {
      std::vector<float> sorted = dur;
      std::nth_element(sorted.begin(), sorted.begin() + sorted.size() / 2, sorted.end());
      const float cut = 0.25f * sorted[sorted.size() / 2];
      for (float d : dur)
        if (d >= cut) {
          dms += d;
          dcalls += 2;
        }
    }
  }
  double sites = 0.0;
  for (int p = 0; p < nprob; ++p) sites += (double)probs[p].lat->g.half * probs[p].nrhs;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  stag_status first_bad = STAG_OK;
  for (int s = 0; s < nslots; ++s) {
    stag_cg_info& o = info[s];
    std::memset(&o, 0, sizeof(o));
    o.iters = iters[s];
    o.restarts = std::max(0, passes[s] - 1);
    o.n_reliable = n_rel[s];
    o.fell_back = fell_back[s];
    o.true_resid = R.h_scal[s].aux;
    o.converged = done_status[s] == STAG_OK;
    o.status = done_status[s];
    o.ms = ms;
    o.dslash_ms = dms;
    o.dslash_calls = dcalls;
    o.dslash_prec = prm.prec;
    o.dslash_sites = sites;
    o.dslash_wg = R.shape.wg;
    o.dslash_rhs = R.shape.r;
    o.dslash_lds = R.shape.lds;
    o.dslash_order = R.shape.order;
    o.dslash_chunks = R.shape.chunks;
    if (first_bad == STAG_OK && done_status[s] != STAG_OK) first_bad = (stag_status)done_status[s];
  }
  if (first_bad != STAG_OK)
    set_error(first_bad == STAG_ERR_NAN ? "a reduction produced NaN/Inf or a non-positive d^dag A d"
                                        : "the solve did not reach the requested true residual");
  return first_bad;
}

}  // namespace stag
