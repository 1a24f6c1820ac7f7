// Launch-shape decisions and their persisted tuning table (the auto-tuner
// of Sec. 4, for the shapes this library offers): per lattice and storage,
// the Dslash shape (one site per work-item, 2- or 4-way direction split)
// and the staple-force shape (one link per work-item or plane split).
//
// Precedence: environment override (HMC_DSLASH_SPLIT, HMC_GFORCE_PLANES) >
// tuned entry > built-in rule measured on MI355X.  HMC_TUNE_DB names a table
// file loaded on first use; hmc_autotune fills and saves entries.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace hmc {

namespace {

using Key = std::tuple<int, int, int, int, int, int>;  // L0..L3, kind, prec

struct Entry {
  int choice;
  double us;
};

struct Table {
  std::mutex mu;
  std::map<Key, Entry> map;
  bool env_loaded = false;
};

Table& table() {
  static Table t;
  return t;
}

Key make_key(const int* L, int kind, int prec) { return Key(L[0], L[1], L[2], L[3], kind, prec); }

const char* kind_name(int kind) { return kind == TUNE_DSLASH ? "dslash" : "gauge_force"; }

bool valid_choice(int kind, int c) { return kind == TUNE_DSLASH ? (c == 1 || c == 2 || c == 4) : (c == 0 || c == 1); }

// Parses "kind L0 L1 L2 L3 prec choice us" lines; others are skipped.
int load_locked(Table& t, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  char line[256];
  int n = 0;
  while (std::fgets(line, sizeof line, f)) {
    char kind[32];
    int L[4], prec, choice;
    double us;
    if (std::sscanf(line, "%31s %d %d %d %d %d %d %lf", kind, &L[0], &L[1], &L[2], &L[3], &prec, &choice, &us) != 8)
      continue;
    int k = std::strcmp(kind, "dslash") == 0 ? TUNE_DSLASH : std::strcmp(kind, "gauge_force") == 0 ? TUNE_GFORCE : -1;
    if (k < 0 || !valid_choice(k, choice) || prec < 0 || prec > 3) continue;
    t.map[make_key(L, k, prec)] = Entry{choice, us};
    ++n;
  }
  std::fclose(f);
  return n;
}

void ensure_env_loaded(Table& t) {
  if (t.env_loaded) return;
  t.env_loaded = true;
  if (const char* p = std::getenv("HMC_TUNE_DB")) load_locked(t, p);
}

int env_int(const char* name) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : -1;
}

}  // namespace

int tune_lookup(const int* L, int kind, int prec) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  ensure_env_loaded(t);
  auto it = t.map.find(make_key(L, kind, prec));
  return it == t.map.end() ? -1 : it->second.choice;
}

void tune_store(const int* L, int kind, int prec, int choice, double us) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  ensure_env_loaded(t);
  t.map[make_key(L, kind, prec)] = Entry{choice, us};
}

int tune_load(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  ensure_env_loaded(t);
  return load_locked(t, path);
}

int tune_save(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  // merge: entries already in the file that this process does not hold are kept
  std::map<Key, Entry> merged;
  {
    Table tmp;
    if (load_locked(tmp, path) >= 0) merged = tmp.map;
  }
  for (const auto& kv : t.map) merged[kv.first] = kv.second;
  const std::string tmp_path = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp_path.c_str(), "w");
  if (!f) return -1;
  std::fprintf(f,
               "# kind L0 L1 L2 L3 prec choice us\n"
               "# dslash: choice 1 = one site per work-item, 2|4 = direction split; us per CG iteration in a solve\n"
               "# gauge_force: choice 0 = one link per work-item, 1 = plane split; us per launch\n");
  for (const auto& kv : merged) {
    const Key& k = kv.first;
    std::fprintf(f, "%s %d %d %d %d %d %d %.3f\n", kind_name(std::get<4>(k)), std::get<0>(k), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), std::get<5>(k), kv.second.choice, kv.second.us);
  }
  std::fclose(f);
  return std::rename(tmp_path.c_str(), path) == 0 ? (int)merged.size() : -1;
}

bool tune_env_forced() { return env_int("HMC_DSLASH_SPLIT") >= 0 || env_int("HMC_GFORCE_PLANES") >= 0; }

int dslash_shape(const LatArg& g, hmc_prec prec) {
  static const int forced = [] {
    const int v = env_int("HMC_DSLASH_SPLIT");
    return v < 0 ? -1 : v == 1 ? 4 : (v == 2 || v == 4) ? v : 1;
  }();
  if (forced > 0) return forced;
  const int t = tune_lookup(g.L, TUNE_DSLASH, prec);
  if (t > 0) return t;
  // measured on MI355X: the 4-way split gains for FP32 arithmetic up to
  // 16^3x32 and loses at 48^3x96; FP64 is even at 16^3x32
  return (prec != HMC_F64 && g.Vh <= (1 << 17)) ? 4 : 1;
}

int gauge_force_shape(const LatArg& g) {
  static const int forced = env_int("HMC_GFORCE_PLANES");
  if (forced >= 0) return forced != 0;
  const int t = tune_lookup(g.L, TUNE_GFORCE, HMC_F64);
  if (t >= 0) return t;
  // measured on MI355X: the plane split is 6% faster at 48^3x96 and 20%
  // slower at 16^3x32
  return g.Vh > (1 << 20) ? 1 : 0;
}

}  // namespace hmc
