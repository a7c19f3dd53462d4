// Autotuner for the Dslash launch shape: workgroup size (sites per workgroup),
// right-hand sides per lane, LDS staging of the x/y neighbour window and the
// tile order (lattice order, or XCD blocks with their number of z blocks per XCD), and, for FP16
// batches of 8k right-hand sides, the time-streaming kernel with its number of time chunks.  Candidates are timed with HIP events on the caller's
// stream on the real buffers of the call; winners are kept per key
// (lattice shapes, right-hand sides, storage precision) in memory and can be saved
// to / loaded from a small JSON file.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "runtime.h"

namespace stag {

namespace {

std::mutex g_mu;
std::map<std::string, DslashShape> g_table;   // tuned or pinned shapes

std::string key_of(const BatchHost& bh, const std::vector<const stag_lattice_s*>& lats, int prec) {
  std::ostringstream k;
  k << "p" << prec << (bh.long12 ? "c" : "");
  for (size_t i = 0; i < lats.size(); ++i) {
    const int* d = lats[i]->dims;
    k << ":" << d[0] << "x" << d[1] << "x" << d[2] << "x" << d[3] << "/" << bh.probs[i].nrhs;
  }
  return k.str();
}

int rhs_divisor(const BatchHost& bh) {
  int r = 8;
  for (const auto& p : bh.probs)
    while (r > 1 && p.nrhs % r) r >>= 1;
  return r;
}

// Without a tuned entry: the XCD z-block order where the lattice allows it (else the lattice order),
// and the best measured shape on the large lattices: 64-site workgroups with up to 4 RHS per lane, or,
// for FP16 with 18-real three-hop links (no third-row rebuild, so 8 RHS fit a lane's registers),
// 128-site workgroups with up to 8.
DslashShape heuristic(const BatchHost& bh, int prec) {
  DslashShape s;
  const bool r8 = prec == P16 && !bh.long12;
  s.r = std::min(rhs_divisor(bh), r8 ? 8 : 4);
  s.wg = r8 && s.r == 8 ? 128 : 64;
  s.order = 1;
  if (!dslash_shape_valid(bh, prec, s)) s.order = 0;
  if (!dslash_shape_valid(bh, prec, s)) s = DslashShape{64, 1, 0, 0};
  return s;
}

}  // namespace

std::string tune_key(const BatchHost& bh, const std::vector<const stag_lattice_s*>& lats, int prec) {
  return key_of(bh, lats, prec);
}

DslashShape lookup_shape(const BatchHost& bh, const std::string& key, int prec) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key);
  if (it != g_table.end()) {
    DslashShape s = it->second;
    s.r = std::min(s.r, rhs_divisor(bh));
    if (!dslash_shape_valid(bh, prec, s)) {  // a loaded entry that does not fit this batch
      s.lds = s.order = 0;
      s.chunks = 1;
    }
    return s;
  }
  return heuristic(bh, prec);
}

void pin_shape(const std::string& key, const DslashShape& s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (s.wg == 0)
    g_table.erase(key);
  else
    g_table[key] = s;
}

bool has_shape(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_table.count(key) != 0;
}

// Time every candidate shape on the batch's Dslash (in_id -> out_id, output parity 1, plain epilogue).
hipError_t tune_batch(const BatchHost& bh, const std::string& key, int prec, hipStream_t st, DslashShape* best_out,
                      std::vector<std::pair<DslashShape, float>>* all, int in_id, int out_id) {
  const int rmax = rhs_divisor(bh);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  DslashShape best{};
  float best_us = 1e30f;
  const int reps = 5;
  std::vector<DslashShape> cands;
  for (int wg : {64, 128, 256})
    for (int r = 1; r <= rmax; r *= 2)
      for (int v = 0; v < 4; ++v) cands.push_back(DslashShape{wg, r, v & 1, v >> 1});
  // thinner XCD z blocks (2, 3, 4 or 6 per XCD) for the shapes without LDS staging
  for (int wg : {64, 128})
    for (int r = 1; r <= rmax; r *= 2)
      for (int c : {2, 3, 4, 6}) cands.push_back(DslashShape{wg, r, 0, 1, c});
  for (int r : {8, 4})
    for (int chunks : {1, 2, 4}) cands.push_back(DslashShape{64, r, 0, 2, chunks});
  for (const DslashShape& sh : cands) {
    if (e != hipSuccess) break;
    if (!dslash_shape_valid(bh, prec, sh)) continue;
    for (int w = 0; w < 2 && e == hipSuccess; ++w)
      e = launch_dslash(bh, prec, EPI_PLAIN, 1, in_id, out_id, 0, 0, 3, sh, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
      e = launch_dslash(bh, prec, EPI_PLAIN, 1, in_id, out_id, 0, 0, 3, sh, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    const float us = 1e3f * ms / reps;
    if (all) all->push_back({sh, us});
    if (us < best_us) {
      best_us = us;
      best = sh;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e == hipSuccess) {
    pin_shape(key, best);
    if (best_out) *best_out = best;
  }
  return e;
}

bool save_table(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ofstream f(path);
  if (!f) return false;
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : g_table) {
    f << "  \"" << kv.first << "\": [" << kv.second.wg << ", " << kv.second.r << ", " << kv.second.lds << ", "
      << kv.second.order << ", " << kv.second.chunks << "]"
      << (++i < g_table.size() ? ",\n" : "\n");
  }
  f << "}\n";
  return (bool)f;
}

// Reads the format save_table writes: one "key": [wg, r, lds, order, chunks] entry per line (lds and
// order may be absent: 0; chunks: 1).
bool load_table(const char* path, int* n_loaded) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  int n = 0;
  std::map<std::string, DslashShape> tmp;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    const size_t b0 = line.find('[', q1);
    if (q1 == std::string::npos || b0 == std::string::npos) return false;
    int wg = 0, r = 0, lds = 0, order = 0, chunks = 1;
    const int got = std::sscanf(line.c_str() + b0, "[%d , %d , %d , %d , %d]", &wg, &r, &lds, &order, &chunks);
    if (got < 2) return false;
    if ((wg != 64 && wg != 128 && wg != 256) || (r != 1 && r != 2 && r != 4 && r != 8) || (lds != 0 && lds != 1) ||
        (order < 0 || order > 2) || chunks < 1 || chunks > 64)
      return false;
    tmp[line.substr(q0 + 1, q1 - q0 - 1)] = DslashShape{wg, r, lds, order, chunks};
    ++n;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : tmp) g_table[kv.first] = kv.second;
  if (n_loaded) *n_loaded = n;
  return true;
}

}  // namespace stag
