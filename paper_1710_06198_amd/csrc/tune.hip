// Kernel variant table.  Several steps of the path have more than one
// correct kernel for a given shape (vector ALU or matrix cores, register
// budget per workgroup).  The launchers ask this table for the shape they
// are about to run; without an entry they use their built-in rule.  The
// table is filled by the autotuner (which times every variant on the
// context's own hierarchy) or loaded from the JSON file it writes.
#include "kernels.h"
#include "tmamg.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

static_assert(TUNE_COARSE_APPLY == TMAMG_TUNE_COARSE_APPLY && TUNE_SAP1 == TMAMG_TUNE_SAP1 &&
                  TUNE_RESTRICT0 == TMAMG_TUNE_RESTRICT0 && TUNE_PROLONG0 == TMAMG_TUNE_PROLONG0 &&
                  TUNE_SAP0 == TMAMG_TUNE_SAP0,
              "variant families must match the public header");

namespace {

struct Entry {
  int variant;
  double ms[TUNE_MAX_VARIANTS];
};

using Key = std::tuple<int, long, long, long>;

std::mutex g_mu;
std::map<Key, Entry> g_table;
int g_count = 0;                    // entries, read without the lock on the launch path
int g_used[TUNE_NFAM] = {};         // variant each family ran last (host side)

const char* const kFamilyNames[TUNE_NFAM] = {"coarse_apply", "sap1", "restrict0", "prolong0", "sap0"};

int family_of(const char* name) {
  for (int f = 0; f < TUNE_NFAM; ++f)
    if (std::strcmp(name, kFamilyNames[f]) == 0) return f;
  return -1;
}

// Minimal reader for the file tune_save writes: one object per entry with
// "family": "<name>", "shape": [a, b, c], "variant": v, in that order.
const char* skip_to(const char* p, const char* tok) {
  const char* q = std::strstr(p, tok);
  return q ? q + std::strlen(tok) : nullptr;
}

}  // namespace

const char* tune_family_name(int family) { return family >= 0 && family < TUNE_NFAM ? kFamilyNames[family] : "?"; }

int tune_get(int family, long a, long b, long c) {
  if (__atomic_load_n(&g_count, __ATOMIC_ACQUIRE) == 0) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(Key(family, a, b, c));
  return it == g_table.end() ? -1 : it->second.variant;
}

void tune_put(int family, long a, long b, long c, int variant, const double* ms, int nms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (variant < 0) {
    g_table.erase(Key(family, a, b, c));
  } else {
    Entry e;
    e.variant = variant;
    for (int k = 0; k < TUNE_MAX_VARIANTS; ++k) e.ms[k] = (ms && k < nms) ? ms[k] : -1.0;
    g_table[Key(family, a, b, c)] = e;
  }
  __atomic_store_n(&g_count, (int)g_table.size(), __ATOMIC_RELEASE);
}

void tune_used(int family, int variant) {
  if (family >= 0 && family < TUNE_NFAM) g_used[family] = variant;
}
int tune_last_used(int family) { return family >= 0 && family < TUNE_NFAM ? g_used[family] : -1; }

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  __atomic_store_n(&g_count, 0, __ATOMIC_RELEASE);
}

int tune_entries() {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_table.size();
}

bool tune_save(const char* path, const char* device) {
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\n  \"format\": \"tmamg-tune-1\",\n  \"device\": \"%s\",\n  \"entries\": [", device ? device : "");
  bool first = true;
  for (const auto& kv : g_table) {
    const Key& k = kv.first;
    const Entry& e = kv.second;
    std::fprintf(f, "%s\n    {\"family\": \"%s\", \"shape\": [%ld, %ld, %ld], \"variant\": %d, \"ms\": [",
                 first ? "" : ",", kFamilyNames[std::get<0>(k)], std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 e.variant);
    bool f2 = true;
    for (int v = 0; v < TUNE_MAX_VARIANTS; ++v) {
      if (e.ms[v] < 0) continue;
      std::fprintf(f, "%s[%d, %.6f]", f2 ? "" : ", ", v, e.ms[v]);
      f2 = false;
    }
    std::fprintf(f, "]}");
    first = false;
  }
  std::fprintf(f, "\n  ]\n}\n");
  return std::fclose(f) == 0;
}

// Returns the number of entries read, or -1 if the file cannot be read or
// holds a malformed entry (then nothing is added).
int tune_load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return -1;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  if (text.find("\"tmamg-tune-1\"") == std::string::npos) return -1;
  struct Row { int fam; long a, b, c; int v; };
  std::vector<Row> rows;
  const char* p = text.c_str();
  while ((p = skip_to(p, "\"family\"")) != nullptr) {
    const char* q = std::strchr(p, '"');
    if (!q) return -1;
    const char* e = std::strchr(q + 1, '"');
    if (!e) return -1;
    const std::string name(q + 1, e - q - 1);
    Row r;
    r.fam = family_of(name.c_str());
    if (r.fam < 0) return -1;
    const char* s = skip_to(e, "\"shape\"");
    if (!s || !(s = std::strchr(s, '['))) return -1;
    char* end = nullptr;
    r.a = std::strtol(s + 1, &end, 10);
    if (!end || *end != ',') return -1;
    r.b = std::strtol(end + 1, &end, 10);
    if (!end || *end != ',') return -1;
    r.c = std::strtol(end + 1, &end, 10);
    if (!end || *end != ']') return -1;
    const char* v = skip_to(end, "\"variant\"");
    if (!v || !(v = std::strchr(v, ':'))) return -1;
    r.v = (int)std::strtol(v + 1, &end, 10);
    if (end == v + 1 || r.v < 0 || r.v >= TUNE_MAX_VARIANTS) return -1;
    rows.push_back(r);
    p = end;
  }
  for (const Row& r : rows) tune_put(r.fam, r.a, r.b, r.c, r.v, nullptr, 0);
  return (int)rows.size();
}
