// Launch-shape and link-form decisions and their persisted tuning table
// (the auto-tuner of Sec. 4, for the choices this library offers): per
// lattice and storage, the Dslash shape (one site per work-item, 2- or
// 4-way direction split), its link streaming, site order and workgroups per
// CU, the staple-force shape (one link per work-item, plane split, or four
// directions of 64 sites per block in the tiled walk), and
// the compact link form of the hop and staple kernels (two rows, or row 0
// and column 2).
//
// Precedence: environment override (HMC_DSLASH_SPLIT, HMC_GFORCE_PLANES,
// HMC_LINK_FORM, HMC_LINK_STREAM, HMC_DSLASH_ORDER, HMC_DSLASH_OCC) > tuned
// entry > built-in rule measured on MI355X.
// HMC_TUNE_DB names a table file loaded on first use; hmc_autotune fills and
// saves entries.
#include <hip/hip_runtime.h>

#include <atomic>
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

// Bumped whenever an entry may have changed (recorded solver launches
// depend on the decisions in force when they were recorded).
std::atomic<uint64_t> g_generation{1};

Table& table() {
  static Table t;
  return t;
}

Key make_key(const int* L, int kind, int prec) { return Key(L[0], L[1], L[2], L[3], kind, prec); }

const char* const kKindNames[] = {"dslash",        "gauge_force",  "dslash_links",    "gauge_force_links",
                                  "dslash_stream", "dslash_order", "dslash_occupancy"};
constexpr int kNumKinds = 7;

const char* kind_name(int kind) { return kKindNames[kind]; }

int kind_of(const char* name) {
  for (int k = 0; k < kNumKinds; ++k)
    if (std::strcmp(name, kKindNames[k]) == 0) return k;
  return -1;
}

bool valid_choice(int kind, int c) {
  switch (kind) {
    case TUNE_DSLASH: return c == 1 || c == 2 || c == 4;
    case TUNE_GFORCE: return c == 0 || c == 1 || c == 2;
    case TUNE_DSLASH_STREAM: return c == 0 || c == 1;
    case TUNE_DSLASH_ORDER: return c >= 0 && c <= kMaxYBlock;
    case TUNE_DSLASH_OCC: return c == 0 || c == 2;
    default: return c == LINK_ROWS2 || c == LINK_ROWCOL;
  }
}

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
    const int k = kind_of(kind);
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
  ++g_generation;
}

int tune_load(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> lk(t.mu);
  ensure_env_loaded(t);
  ++g_generation;
  return load_locked(t, path);
}

uint64_t tune_generation() { return g_generation.load(); }

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
               "# gauge_force: choice 0 = one link per work-item, 1 = plane split, 2 = four directions of 64 sites per "
               "block; us per launch\n"
               "# dslash_links, gauge_force_links: reals read per SU(3) link, 12 = two rows, 10 = row 0 and column 2\n"
               "# dslash_stream: 1 = non-temporal link loads and output stores\n"
               "# dslash_order: 1 = tiled site order (one site per work-item shape), n >= 2 = tiled in y-blocks of n "
               "64-site chunks\n"
               "# dslash_occupancy: workgroups per CU of the tiled order, 2 = at most two, 0 = as registers allow\n");
  for (const auto& kv : merged) {
    const Key& k = kv.first;
    std::fprintf(f, "%s %d %d %d %d %d %d %.3f\n", kind_name(std::get<4>(k)), std::get<0>(k), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), std::get<5>(k), kv.second.choice, kv.second.us);
  }
  std::fclose(f);
  return std::rename(tmp_path.c_str(), path) == 0 ? (int)merged.size() : -1;
}

bool tune_env_forced() {
  return env_int("HMC_DSLASH_SPLIT") >= 0 || env_int("HMC_GFORCE_PLANES") >= 0 || env_int("HMC_LINK_FORM") >= 0 ||
         env_int("HMC_LINK_STREAM") >= 0 || env_int("HMC_DSLASH_ORDER") >= 0 || env_int("HMC_DSLASH_OCC") >= 0;
}

namespace {
// HMC_LINK_FORM: 18 = all entries even on SU(3) links, 12, 10; else unset.
int forced_link_form() {
  static const int forced = [] {
    const int v = env_int("HMC_LINK_FORM");
    return (v == LINK_FULL || v == LINK_ROWS2 || v == LINK_ROWCOL) ? v : -1;
  }();
  return forced;
}
}  // namespace

int dslash_link_form(const LatArg& g, hmc_prec prec) {
  if (forced_link_form() > 0) return forced_link_form();
  const int t = tune_lookup(g.L, TUNE_DSLASH_LINKS, prec);
  if (t > 0) return t;
  // measured on MI355X: the 10-real form's reconstruction lengthens each
  // hop, which costs at 16^3x32 (latency-bound) and pays at 48^3x96
  return g.Vh >= (1 << 20) ? LINK_ROWCOL : LINK_ROWS2;
}

bool dslash_link_stream(const LatArg& g, hmc_prec prec) {
  static const int forced = env_int("HMC_LINK_STREAM");
  if (forced >= 0) return forced != 0;
  const int t = tune_lookup(g.L, TUNE_DSLASH_STREAM, prec);
  if (t >= 0) return t != 0;
  // measured on MI355X: 17% faster FP64 Dslash at 48^3x96, 30% slower at
  // 16^3x32, whose fields stay in the last-level cache between launches
  return g.Vh >= (1 << 20);
}

int dslash_tiled_order(const LatArg& g, hmc_prec prec) {
  if (!tiled_order_valid(g)) return 0;
  static const int forced = env_int("HMC_DSLASH_ORDER");
  // an order the lattice does not admit falls back to whole z-planes
  if (forced >= 0) return forced == 0 ? 0 : tiled_order_valid(g, forced) ? forced : 1;
  const int t = tune_lookup(g.L, TUNE_DSLASH_ORDER, prec);
  if (t >= 0) return t == 0 ? 0 : tiled_order_valid(g, t) ? t : 1;
  return 0;
}

int dslash_tiled_occupancy(const LatArg& g, hmc_prec prec) {
  static const int forced = env_int("HMC_DSLASH_OCC");
  if (forced >= 0) return forced == 0 ? 0 : 2;
  const int t = tune_lookup(g.L, TUNE_DSLASH_OCC, prec);
  if (t >= 0) return t;
  return 2;
}

int staple_link_form(const LatArg& g) {
  if (forced_link_form() > 0) return forced_link_form();
  const int t = tune_lookup(g.L, TUNE_GFORCE_LINKS, HMC_F64);
  if (t > 0) return t;
  // measured on MI355X: faster at 16^3x32 and 48^3x96
  return LINK_ROWCOL;
}

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

bool exp_update_stream(const LatArg& g) {
  static const int forced = env_int("HMC_EXP_STREAM");
  if (forced >= 0) return forced != 0;
  // measured on MI355X: 16^3x32 27.4 -> 29.8 us (the fields stay in the
  // last-level cache between launches, which the hints bypass); 24^3x48
  // 156 -> 144 us, 32^4 270 -> 250 us; 48^3x96 2.56-2.58 ms either way
  return g.Vh >= (1 << 18);
}

bool fermion_force_stream(const LatArg& g) {
  static const int forced = env_int("HMC_FF_STREAM");
  if (forced >= 0) return forced != 0;
  // measured on MI355X: 24^3x48 174 -> 156 us, 48^3x96 2.99 -> 2.90 ms;
  // 16^3x32 31.6 against 31.7 us
  return g.Vh >= (1 << 18);
}

bool gauge_force_stream(const LatArg& g) {
  static const int forced = env_int("HMC_GF_STREAM");
  if (forced >= 0) return forced != 0;
  // measured on MI355X (site-blocked staple force): 24^3x48 321 -> 295 us,
  // 48^3x96 4.65 -> 4.57 ms
  return g.Vh >= (1 << 18);
}

int plaquette_shape(const LatArg&) {
  static const int forced = env_int("HMC_PLAQ_PAIRS");
  if (forced >= 0) return forced == 0 ? 0 : 1;
  // measured on MI355X: 1.78 -> 1.36 ms at 48^3x96, 26.5 -> 21.3 us at 16^3x32
  return 1;
}

int plaquette_link_form(const LatArg& g) {
  static const int forced = env_int("HMC_PLAQ_FORM");
  if (forced == LINK_ROWS2 || forced == LINK_ROWCOL) return forced;
  // measured on MI355X (plane-paired sum): two rows 1.33 ms against 1.69 ms
  // with row 0 + column 2 at 48^3x96, 21.4 against 29.6 us at 16^3x32 (the
  // reconstruction lengthens the latency-bound chain); the per-site form
  // follows the staple force
  return plaquette_shape(g) == 1 ? (int)LINK_ROWS2 : staple_link_form(g);
}


int gauge_force_shape(const LatArg& g) {
  static const int forced = env_int("HMC_GFORCE_PLANES");
  if (forced >= 0) return forced == 0 ? 0 : forced == 2 ? 2 : 1;
  const int t = tune_lookup(g.L, TUNE_GFORCE, HMC_F64);
  if (t >= 0) return t;
  // measured on MI355X: four directions per block in the tiled walk are
  // 27% faster than one link per work-item at 48^3x96 and 13% faster at
  // 16^3x32 (the plane split: 6% slower and 20% slower)
  return 2;
}

}  // namespace hmc
