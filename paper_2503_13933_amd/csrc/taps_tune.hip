// Timing autotuner of the batched driver: the row split of the load-Gram
// work items (lgram_rows, a tile parameter of the persistent load-Gram
// kernel) and how many sweeps one captured HIP graph holds (0 = launches from
// the host).  The row splits are timed with host launches first, then the
// graph lengths with the best split (a coordinate search: eight timed runs).
// Candidates are timed on the caller's batch with HIP events; the factors
// are saved and restored around the trials.  Choices are cached in a small
// JSON file keyed by the batch shape, one entry per line:
//   {
//     "B=256;D=4;M=40;solver=1;s=2,2,2,2;n=512,512,128,257;R=257,1,1,257;K=2,2,2,2": {"graph_sweeps": 1, "lgram_rows": 512, "ms_per_sweep": 151.2},
//     ...
//   }
#include "taps_internal.hpp"

#include <algorithm>
#include <fstream>
#include <sstream>

namespace {

constexpr int kCandidates[4] = {0, 1, 2, 4};
constexpr int kRowCandidates[4] = {128, 256, 512, 1024};
constexpr int kTimedSweeps = 4;

std::string shape_key(int B, const taps_problem_t* probs, int solver) {
  const taps_problem_t& p0 = probs[0];
  std::ostringstream k;
  k << "B=" << B << ";D=" << p0.D << ";M=" << p0.M << ";solver=" << solver << ";s=";
  for (int d = 0; d < p0.D; ++d) k << (d ? "," : "") << p0.s[d];
  const char* tags[3] = {";n=", ";R=", ";K="};
  for (int f = 0; f < 3; ++f) {
    k << tags[f];
    for (int d = 0; d < p0.D; ++d) {
      int mx = 0;
      for (int b = 0; b < B; ++b)
        mx = std::max(mx, f == 0 ? probs[b].n[d] : f == 1 ? probs[b].R_cols[d] : probs[b].n_kinds[d]);
      k << (d ? "," : "") << mx;
    }
  }
  return k.str();
}

// Entry lines of the cache file (everything between the outer braces).
std::vector<std::string> read_entries(const char* path) {
  std::vector<std::string> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t q = line.find('"');
    if (q == std::string::npos) continue;
    out.push_back(line.substr(q));
    if (!out.back().empty() && out.back().back() == ',') out.back().pop_back();
  }
  return out;
}

bool lookup(const std::vector<std::string>& entries, const std::string& key, int* graph_sweeps, int* lgram_rows) {
  const std::string head = "\"" + key + "\"";
  for (const auto& e : entries) {
    if (e.compare(0, head.size(), head) != 0) continue;
    const size_t g = e.find("\"graph_sweeps\":");
    const size_t r = e.find("\"lgram_rows\":");
    if (g == std::string::npos || r == std::string::npos) continue;
    *graph_sweeps = std::atoi(e.c_str() + g + 15);
    *lgram_rows = std::atoi(e.c_str() + r + 13);
    return true;
  }
  return false;
}

bool write_entries(const char* path, const std::vector<std::string>& entries) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return false;
  f << "{\n";
  for (size_t i = 0; i < entries.size(); ++i) f << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  f << "}\n";
  return bool(f);
}

}  // namespace

using namespace taps;

extern "C" taps_status taps_autotune(taps_handle_t h, int32_t B, const taps_problem_t* probs, double* const* d_U,
                                     const char* cache_path, taps_tuning_t* chosen, double* ms_per_sweep,
                                     hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (B < 1 || !probs || !d_U || !chosen) return fail(h, TAPS_ERR_INVALID, "bad autotune arguments");
  for (int b = 0; b < B; ++b) TAPS_TRY(check_problem(h, &probs[b]));
  const std::string key = shape_key(B, probs, h->tune.solver);
  std::vector<std::string> entries;
  if (cache_path) {
    entries = read_entries(cache_path);
    int K = 0, rows = 0;
    if (lookup(entries, key, &K, &rows) && K >= 0 && K <= 16 && rows >= 16 && rows <= 4096 && rows % 16 == 0) {
      h->tune.graph_sweeps = K;
      h->tune.lgram_rows = rows;
      *chosen = h->tune;
      if (ms_per_sweep)
        for (int c = 0; c < 8; ++c) ms_per_sweep[c] = -1.0;
      return TAPS_OK;
    }
  }
  if (h->prof.on) return fail(h, TAPS_ERR_INVALID, "autotune needs kernel timing disabled");
  // save the factors
  const int D = probs[0].D, M = probs[0].M;
  size_t total = 0;
  for (int b = 0; b < B; ++b)
    for (int d = 0; d < D; ++d) total += size_t(probs[b].n[d]) * M;
  double* saved = nullptr;
  TAPS_HIP(h, hipMalloc(&saved, total * 8));
  auto copy_all = [&](bool save) -> taps_status {
    size_t off = 0;
    for (int b = 0; b < B; ++b)
      for (int d = 0; d < D; ++d) {
        const size_t n = size_t(probs[b].n[d]) * M;
        double* u = d_U[size_t(b) * D + d];
        TAPS_HIP(h, hipMemcpyAsync(save ? saved + off : u, save ? u : saved + off, n * 8, hipMemcpyDeviceToDevice,
                                   stream));
        off += n;
      }
    return TAPS_OK;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<int32_t> sw(B);
  std::vector<double> rho(B);
  double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // row splits 128..1024, then graph lengths 0..4
  const taps_tuning_t before = h->tune;
  taps_status st = copy_all(true);
  if (st == TAPS_OK && hipEventCreate(&e0) != hipSuccess) st = fail(h, TAPS_ERR_HIP, "event creation failed");
  if (st == TAPS_OK && hipEventCreate(&e1) != hipSuccess) st = fail(h, TAPS_ERR_HIP, "event creation failed");
  auto trial = [&](double* out) {
    // untimed run (captures a graph), then the timed one from the same factors
    st = copy_all(false);
    if (st == TAPS_OK) st = taps_als_batched(h, B, probs, d_U, 0.0, 0.0, kTimedSweeps, sw.data(), rho.data(), nullptr, stream);
    if (st == TAPS_OK) st = copy_all(false);
    if (st == TAPS_OK && hipEventRecord(e0, stream) != hipSuccess) st = fail(h, TAPS_ERR_HIP, "event record failed");
    if (st == TAPS_OK) st = taps_als_batched(h, B, probs, d_U, 0.0, 0.0, kTimedSweeps, sw.data(), rho.data(), nullptr, stream);
    if (st == TAPS_OK && hipEventRecord(e1, stream) != hipSuccess) st = fail(h, TAPS_ERR_HIP, "event record failed");
    float t = 0.0f;
    if (st == TAPS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      st = fail(h, TAPS_ERR_HIP, "event timing failed");
    *out = double(t) / kTimedSweeps;
  };
  // the smallest candidate index within 3 % of the fastest
  auto pick_of = [](const double* v) {
    const double best = *std::min_element(v, v + 4);
    for (int c = 0; c < 4; ++c)
      if (v[c] <= 1.03 * best) return c;
    return 3;
  };
  h->tune.graph_sweeps = 0;
  for (int c = 0; c < 4 && st == TAPS_OK; ++c) {
    h->tune.lgram_rows = kRowCandidates[c];
    trial(&ms[c]);
  }
  int pick_rows = 1;
  if (st == TAPS_OK) {
    // rows: the fastest (no preference for small values)
    pick_rows = int(std::min_element(ms, ms + 4) - ms);
    h->tune.lgram_rows = kRowCandidates[pick_rows];
  }
  for (int c = 0; c < 4 && st == TAPS_OK; ++c) {
    h->tune.graph_sweeps = kCandidates[c];
    trial(&ms[4 + c]);
  }
  if (st == TAPS_OK) st = copy_all(false);
  if (st == TAPS_OK && hipStreamSynchronize(stream) != hipSuccess) st = fail(h, TAPS_ERR_HIP, "synchronisation failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(saved);
  if (st != TAPS_OK) {
    h->tune = before;
    return st;
  }
  const int pick = pick_of(ms + 4);
  h->tune.graph_sweeps = kCandidates[pick];
  h->tune.lgram_rows = kRowCandidates[pick_rows];
  *chosen = h->tune;
  if (ms_per_sweep)
    for (int c = 0; c < 8; ++c) ms_per_sweep[c] = ms[c];
  if (cache_path) {
    std::ostringstream e;
    e << "\"" << key << "\": {\"graph_sweeps\": " << kCandidates[pick] << ", \"lgram_rows\": "
      << kRowCandidates[pick_rows] << ", \"ms_per_sweep\": " << ms[4 + pick] << "}";
    entries.push_back(e.str());
    if (!write_entries(cache_path, entries)) return fail(h, TAPS_ERR_INVALID, "cannot write %s", cache_path);
  }
  return TAPS_OK;
}
