// Process-wide table of tuned pair-sum launch shapes, and its text file form.  Host code only: the
// timing runs that fill it live with the operator in mfs_api.hip.
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "mfs_internal.h"

namespace mfs {
namespace {

using TuneKey = std::tuple<int, int, int, int>;  // dim, variant, R, floor(log2 N)

std::mutex g_mu;
std::map<TuneKey, LaunchShape> g_table;

int log2_floor(int64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

bool valid(int dim, int variant, int R, int lg, LaunchShape v) {
  return (dim == 2 || dim == 3) && variant >= kTunePairF64 && variant <= kTunePairMfma && R >= 1 && lg >= 0 &&
         lg < 63 && v.nchunks >= 1 && v.nchunks <= kTuneMaxChunks && (v.rt == 0 || v.rt == 1 || v.rt == 2 || v.rt == 4) &&
         v.sym >= -1 && v.sym <= 1;
}

constexpr const char* kHeader = "mfs-tune 2";

}  // namespace

bool tune_lookup(int dim, int variant, int R, int64_t N, LaunchShape* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(TuneKey{dim, variant, R, log2_floor(N)});
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(int dim, int variant, int R, int64_t N, LaunchShape v) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[TuneKey{dim, variant, R, log2_floor(N)}] = v;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

int64_t tune_size() {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int64_t)g_table.size();
}

// One line per entry: dim variant R log2N nchunks rt sym, after a header line.
bool tune_save(const char* path, std::string* err) {
  std::map<TuneKey, LaunchShape> copy;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    copy = g_table;
  }
  FILE* f = std::fopen(path, "w");
  if (!f) {
    *err = std::string("cannot open ") + path + " for writing";
    return false;
  }
  bool ok = std::fprintf(f, "%s\n", kHeader) > 0;
  for (const auto& [k, v] : copy)
    ok = ok && std::fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                            std::get<3>(k), v.nchunks, v.rt, v.sym) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) *err = std::string("write to ") + path + " failed";
  return ok;
}

// All or nothing: a malformed file leaves the table as it was.
bool tune_load(const char* path, std::string* err) {
  FILE* f = std::fopen(path, "r");
  if (!f) {
    *err = std::string("cannot open ") + path;
    return false;
  }
  char head[32] = {0};
  const bool head_ok = std::fgets(head, sizeof head, f) && std::string(head).rfind(kHeader, 0) == 0;
  std::map<TuneKey, LaunchShape> add;
  int line = 1;
  bool ok = head_ok;
  if (!head_ok) *err = std::string(path) + ": not a launch-shape file (missing header)";
  while (ok) {
    int dim, variant, R, lg, nch, rt, sym;
    const int got = std::fscanf(f, "%d %d %d %d %d %d %d", &dim, &variant, &R, &lg, &nch, &rt, &sym);
    if (got == EOF) break;
    ++line;
    if (got != 7 || !valid(dim, variant, R, lg, LaunchShape{nch, rt, sym})) {
      *err = std::string(path) + ": bad entry on line " + std::to_string(line);
      ok = false;
      break;
    }
    add[TuneKey{dim, variant, R, lg}] = LaunchShape{nch, rt, sym};
  }
  std::fclose(f);
  if (!ok) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& [k, v] : add) g_table[k] = v;
  return true;
}

}  // namespace mfs
