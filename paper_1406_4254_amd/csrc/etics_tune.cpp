// etics_tune.cpp -- tile plans chosen by the autotuner.
//
// The coefficient kernels take their tile shape from a plan (particles per tile,
// particle groups per tile, stream copies, workgroups per CU, outer products on the
// vector ALUs or the matrix cores; for batched systems also the particles per work unit
// and the force workgroups per unit).  make_coeff_plan
// derives a plan from fixed rules; this table holds plans measured to be faster on
// the device by the project's tuner (paper_1406_4254_amd/tune.py), keyed by
// (batched, nmax, lmax, precision, basis) and the particle count they were tuned at.
// A lookup takes the entry of the same key whose particle count is nearest in log2,
// within a factor of 8; otherwise the fixed rules apply.  Every tuned value is checked
// against the kernel's limits by make_coeff_plan before it is used, so a bad file can
// only fall back to the fixed rules.
//
// The table is filled from a JSON file on first use: $ETICS_TUNING_FILE if set,
// otherwise etics_tuning.json next to libetics.so (absent: fixed rules only).  The
// file holds {"plans": [{"batched": 0, "nmax": 10, ..., "nw": 4, "tp": 64, ...}, ...]};
// other keys and string values are ignored.
#include <dlfcn.h>

#include <cctype>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "etics_internal.hpp"

namespace etics {

namespace {

struct Entry {
  int key[5];  // batched, nmax, lmax, prec, basis
  int64_t n;
  TunedParams t;
};

std::mutex g_mu;
std::vector<Entry> g_tab;
bool g_loaded = false;  // the automatic load has run (or the table was set explicitly)

// ------------------------------------------------------------------ tiny JSON reader
// Enough JSON for the tuning file: objects, arrays, strings, numbers, literals.  Every
// object that holds a numeric "nmax" is taken as one plan (its numeric members by
// name); parsing stops with false on malformed input.
struct Reader {
  const char* p;
  const char* e;
  std::vector<std::map<std::string, double>> plans;

  void ws() {
    while (p < e && std::isspace(static_cast<unsigned char>(*p))) ++p;
  }
  bool str(std::string* out) {
    if (p >= e || *p != '"') return false;
    ++p;
    std::string s;
    while (p < e && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= e) return false;
      }
      s.push_back(*p++);
    }
    if (p >= e) return false;
    ++p;
    if (out) *out = s;
    return true;
  }
  bool num(double* out) {
    char* end = nullptr;
    const double v = std::strtod(p, &end);
    if (end == p || end > e) return false;
    p = end;
    *out = v;
    return true;
  }
  bool value(int depth, std::map<std::string, double>* into, const std::string& name) {
    if (depth > 32) return false;
    ws();
    if (p >= e) return false;
    if (*p == '{') return object(depth + 1);
    if (*p == '[') {
      ++p;
      ws();
      if (p < e && *p == ']') {
        ++p;
        return true;
      }
      while (true) {
        if (!value(depth + 1, nullptr, "")) return false;
        ws();
        if (p < e && *p == ',') {
          ++p;
          continue;
        }
        if (p < e && *p == ']') {
          ++p;
          return true;
        }
        return false;
      }
    }
    if (*p == '"') return str(nullptr);
    for (const char* lit : {"true", "false", "null"}) {
      const size_t k = std::strlen(lit);
      if (size_t(e - p) >= k && std::strncmp(p, lit, k) == 0) {
        p += k;
        return true;
      }
    }
    double v;
    if (!num(&v)) return false;
    if (into && !name.empty()) (*into)[name] = v;
    return true;
  }
  bool object(int depth) {
    ++p;  // '{'
    std::map<std::string, double> members;
    ws();
    if (p < e && *p == '}') {
      ++p;
      return true;
    }
    while (true) {
      ws();
      std::string k;
      if (!str(&k)) return false;
      ws();
      if (p >= e || *p != ':') return false;
      ++p;
      if (!value(depth, &members, k)) return false;
      ws();
      if (p < e && *p == ',') {
        ++p;
        continue;
      }
      if (p < e && *p == '}') {
        ++p;
        break;
      }
      return false;
    }
    if (members.count("nmax")) plans.push_back(members);
    return true;
  }
};

bool fits_int(double v) { return std::isfinite(v) && v >= INT_MIN && v <= INT_MAX && v == std::floor(v); }

int parse_plans(const std::string& text, std::vector<Entry>* out) {
  Reader r{text.data(), text.data() + text.size(), {}};
  if (!r.value(0, nullptr, "")) return -1;
  static const char* kKey[5] = {"batched", "nmax", "lmax", "prec", "basis"};
  static const char* kPar[7] = {"nw", "tp", "streams", "grid_mult", "unit", "split", "phase2"};
  for (const auto& m : r.plans) {
    Entry en{};
    bool ok = true;
    for (int i = 0; i < 5 && ok; ++i) {
      auto it = m.find(kKey[i]);
      double v = it == m.end() ? 0.0 : it->second;  // absent batched/basis: 0
      if (it == m.end() && (i == 1 || i == 2 || i == 3)) ok = false;
      if (!fits_int(v)) ok = false;
      en.key[i] = int(v);
    }
    auto itn = m.find("n");
    if (itn == m.end() || !(itn->second >= 1.0) || !(itn->second < 9.0e18)) ok = false;
    if (ok) en.n = int64_t(itn->second);
    int* par[7] = {&en.t.nw, &en.t.tp, &en.t.streams, &en.t.grid_mult, &en.t.unit, &en.t.split, &en.t.phase2};
    for (int i = 0; i < 7 && ok; ++i) {
      auto it = m.find(kPar[i]);
      const double v = it == m.end() ? 0.0 : it->second;  // 0 = keep the fixed rule
      if (!fits_int(v)) ok = false;
      *par[i] = int(v);
    }
    if (ok) out->push_back(en);
  }
  return int(out->size());
}

int load_file_locked(const char* path, bool quiet) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    if (!quiet) set_error(std::string("etics_tuning_load: cannot open ") + path);
    return quiet ? 0 : ETICS_EINVAL;
  }
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (size_t(16) << 20)) text.append(buf, k);
  std::fclose(f);
  std::vector<Entry> tab;
  const int cnt = parse_plans(text, &tab);
  if (cnt < 0) {
    if (!quiet) set_error(std::string("etics_tuning_load: malformed JSON in ") + path);
    return quiet ? 0 : ETICS_EINVAL;
  }
  g_tab = tab;
  return cnt;
}

std::string default_path() {
  Dl_info info{};
  if (dladdr(reinterpret_cast<void*>(&default_path), &info) == 0 || !info.dli_fname) return "";
  std::string so = info.dli_fname;
  const size_t slash = so.rfind('/');
  return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/etics_tuning.json";
}

void ensure_loaded_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* env = std::getenv("ETICS_TUNING_FILE");
  const std::string path = env && *env ? std::string(env) : default_path();
  if (!path.empty()) (void)load_file_locked(path.c_str(), true);
}

}  // namespace

bool tuned_lookup(int batched, int nmax, int lmax, int prec, int basis, int64_t n, TunedParams* out) {
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded_locked();
  const int key[5] = {batched, nmax, lmax, prec, basis};
  const double ln = std::log2(double(n > 0 ? n : 1));
  double best = 3.0 + 1e-9;  // within a factor of 8
  bool found = false;
  for (const Entry& e : g_tab) {
    if (std::memcmp(e.key, key, sizeof key) != 0) continue;
    const double d = std::fabs(std::log2(double(e.n)) - ln);
    if (d <= best) {
      best = d;
      *out = e.t;
      found = true;
    }
  }
  return found;
}

}  // namespace etics

using namespace etics;

extern "C" {

int etics_tuning_load(const char* path) {
  if (!path) {
    set_error("etics_tuning_load: path is NULL");
    return ETICS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  g_loaded = true;
  return load_file_locked(path, false);
}

int etics_tuning_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_loaded = true;
  g_tab.clear();
  return ETICS_OK;
}

int etics_tuning_set(int batched, int nmax, int lmax, int precision, int basis, int64_t n,
                     const int* params, int nparams) {
  if (!params || nparams != 7 || n < 1 || (batched != 0 && batched != 1)) {
    set_error("etics_tuning_set: need 7 parameters, n >= 1 and batched 0 or 1");
    return ETICS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  ensure_loaded_locked();
  Entry en{{batched, nmax, lmax, precision, basis}, n,
           {params[0], params[1], params[2], params[3], params[4], params[5], params[6]}};
  for (Entry& e : g_tab)
    if (std::memcmp(e.key, en.key, sizeof en.key) == 0 && e.n == n) {
      e = en;
      return ETICS_OK;
    }
  g_tab.push_back(en);
  return ETICS_OK;
}

}  // extern "C"
