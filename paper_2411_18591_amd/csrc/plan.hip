// Plan table and its file format (host code).
//
// File format, one record per line, '#' starts a comment line:
//   toprop-plan 2                                   (first line, exactly)
//   <c64|c128> <ly> <lx> <col_variant> <chunk_mb> <row_fpb> <us>
// ly, lx: powers of two in [8, 8192]; col_variant in [0, kColVariants);
// chunk_mb in [1, 65536]; row_fpb in [0, 8] (0: automatic); us finite and
// >= 0.  Duplicate keys are an error.  Files of version 1 (the same records
// without row_fpb) are read with row_fpb = 0; files are written as version 2.
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <istream>
#include <sstream>
#include <tuple>

#include "launch.hpp"
#include "plan.hpp"

namespace toprop {
namespace {

using Key = std::tuple<int, int, int>;
std::mutex g_plan_mutex;
std::map<Key, PlanEntry> g_plans;
bool g_env_loaded = false;

const char* kHeader = "toprop-plan 2";
const char* kHeaderV1 = "toprop-plan 1";

bool pow2_len(int n) { return n >= kMinLen && n <= kMaxLen && (n & (n - 1)) == 0; }

// Strict integer parse of a whole token.
bool parse_int(const std::string& t, int* v) {
  if (t.empty() || t.size() > 10) return false;
  char* end = nullptr;
  errno = 0;
  long x = strtol(t.c_str(), &end, 10);
  if (errno || *end != '\0' || x < -2147483647L || x > 2147483647L) return false;
  *v = (int)x;
  return true;
}

bool parse_double(const std::string& t, double* v) {
  if (t.empty()) return false;
  char* end = nullptr;
  errno = 0;
  double x = strtod(t.c_str(), &end);
  if (errno || *end != '\0' || !std::isfinite(x)) return false;
  *v = x;
  return true;
}

// Parses a whole plan file into *out; returns false with the reason in *err.
bool parse_plan(std::istream& in, const char* name, std::map<Key, PlanEntry>* out, std::string* err) {
  std::string line;
  int ln = 0;
  int fields = 7;  // per record: 7 in version 2, 6 in version 1
  char buf[256];
  while (std::getline(in, line)) {
    ++ln;
    if (ln == 1) {
      if (line == kHeaderV1) {
        fields = 6;
      } else if (line != kHeader) {
        snprintf(buf, sizeof buf, "%s: line 1 is not the header '%s' (or '%s')", name, kHeader, kHeaderV1);
        *err = buf;
        return false;
      }
      continue;
    }
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string tok[8];
    int n = 0;
    while (n < 8 && (ls >> tok[n])) ++n;
    if (n != fields) {
      snprintf(buf, sizeof buf, "%s: line %d has %s %d fields", name, ln, n < fields ? "fewer than" : "more than",
               fields);
      *err = buf;
      return false;
    }
    const int dt = tok[0] == "c64" ? 0 : (tok[0] == "c128" ? 1 : -1);
    PlanEntry e;
    int ly, lx;
    e.row_fpb = 0;
    const bool fpb_ok = fields == 6 || parse_int(tok[5], &e.row_fpb);
    if (dt < 0 || !parse_int(tok[1], &ly) || !parse_int(tok[2], &lx) || !parse_int(tok[3], &e.col_variant) ||
        !parse_int(tok[4], &e.chunk_mb) || !fpb_ok || !parse_double(tok[fields - 1], &e.us)) {
      snprintf(buf, sizeof buf, "%s: line %d: malformed record", name, ln);
      *err = buf;
      return false;
    }
    std::string why;
    if (!plan_entry_valid(dt, ly, lx, e, &why)) {
      snprintf(buf, sizeof buf, "%s: line %d: ", name, ln);
      *err = buf + why;
      return false;
    }
    if (!out->emplace(Key(dt, ly, lx), e).second) {
      snprintf(buf, sizeof buf, "%s: line %d: duplicate entry for %s %dx%d", name, ln, tok[0].c_str(), ly, lx);
      *err = buf;
      return false;
    }
  }
  if (ln == 0) {
    *err = std::string(name) + ": empty file (no header)";
    return false;
  }
  return true;
}

void load_env_locked() {
  if (g_env_loaded) return;
  g_env_loaded = true;
  const std::string& p = plan_env_path();
  if (p.empty()) return;
  std::ifstream f(p);
  if (!f) return;  // no cache yet
  std::map<Key, PlanEntry> tmp;
  std::string err;
  if (parse_plan(f, p.c_str(), &tmp, &err)) g_plans.insert(tmp.begin(), tmp.end());
}

}  // namespace

const std::string& plan_env_path() {
  static const std::string p = [] {
    const char* s = getenv("TOPROP_PLAN_CACHE");
    return std::string(s ? s : "");
  }();
  return p;
}

bool plan_entry_valid(int dtype, int ly, int lx, const PlanEntry& e, std::string* err) {
  char buf[160];
  if (dtype != 0 && dtype != 1) {
    snprintf(buf, sizeof buf, "dtype %d is not complex64 (0) or complex128 (1)", dtype);
  } else if (!pow2_len(ly) || !pow2_len(lx)) {
    snprintf(buf, sizeof buf, "padded grid %dx%d is not powers of two in [%d, %d]", ly, lx, kMinLen, kMaxLen);
  } else if (e.col_variant < 0 || e.col_variant >= kColVariants) {
    snprintf(buf, sizeof buf, "column variant %d is outside [0, %d)", e.col_variant, kColVariants);
  } else if (e.chunk_mb < 1 || e.chunk_mb > kPlanMaxChunkMb) {
    snprintf(buf, sizeof buf, "chunk size %d MiB is outside [1, %d]", e.chunk_mb, kPlanMaxChunkMb);
  } else if (e.row_fpb < 0 || e.row_fpb > kPlanMaxRowFpb) {
    snprintf(buf, sizeof buf, "row fields per workgroup %d is outside [0, %d]", e.row_fpb, kPlanMaxRowFpb);
  } else if (!std::isfinite(e.us) || e.us < 0) {
    snprintf(buf, sizeof buf, "time %g is not a finite non-negative number", e.us);
  } else {
    return true;
  }
  if (err) *err = buf;
  return false;
}

bool plan_lookup(int dtype, int ly, int lx, PlanEntry* e) {
  std::lock_guard<std::mutex> lk(g_plan_mutex);
  load_env_locked();
  auto it = g_plans.find(Key(dtype, ly, lx));
  if (it == g_plans.end()) return false;
  *e = it->second;
  return true;
}

void plan_store(int dtype, int ly, int lx, const PlanEntry& e) {
  std::lock_guard<std::mutex> lk(g_plan_mutex);
  load_env_locked();
  g_plans[Key(dtype, ly, lx)] = e;
}

void plan_clear() {
  std::lock_guard<std::mutex> lk(g_plan_mutex);
  g_env_loaded = true;  // a cleared table stays empty until loaded again
  g_plans.clear();
}

int plan_count() {
  std::lock_guard<std::mutex> lk(g_plan_mutex);
  load_env_locked();
  return (int)g_plans.size();
}

int plan_load_file(const char* path, std::string* err) {
  std::ifstream f(path);
  if (!f) {
    *err = std::string("cannot open plan file ") + path;
    return -1;
  }
  std::map<Key, PlanEntry> tmp;
  if (!parse_plan(f, path, &tmp, err)) return -1;
  std::lock_guard<std::mutex> lk(g_plan_mutex);
  g_env_loaded = true;
  for (auto& kv : tmp) g_plans[kv.first] = kv.second;
  return 0;
}

int plan_save_file(const char* path, std::string* err) {
  std::map<Key, PlanEntry> snap;
  {
    std::lock_guard<std::mutex> lk(g_plan_mutex);
    load_env_locked();
    snap = g_plans;
  }
  // write to a temporary file, then rename: a reader never sees half a file
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) {
    *err = std::string("cannot write plan file ") + tmp;
    return -1;
  }
  fprintf(f, "%s\n# dtype ly lx col_variant chunk_mb row_fpb us\n", kHeader);
  for (auto& kv : snap)
    fprintf(f, "%s %d %d %d %d %d %.3f\n", std::get<0>(kv.first) ? "c128" : "c64", std::get<1>(kv.first),
            std::get<2>(kv.first), kv.second.col_variant, kv.second.chunk_mb, kv.second.row_fpb, kv.second.us);
  const bool bad = ferror(f) != 0;
  if (fclose(f) != 0 || bad) {
    remove(tmp.c_str());
    *err = std::string("error writing plan file ") + tmp;
    return -1;
  }
  if (rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    *err = std::string("cannot replace plan file ") + path;
    return -1;
  }
  return 0;
}

}  // namespace toprop
