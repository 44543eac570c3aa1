// Size-class tuning cache of the INT8 product: for a size class (the
// device's architecture, scheme, requested form, ceil(log2) of m, n and k,
// and the slice count in steps of 8) the band width, the work-item target
// that sets the contraction chunks, and (for MPCG_AUTO) the 3M or 4M form
// that mpcg_autotune measured fastest.  Exact-scheme bits do not depend on
// any of these choices.  The cache is a JSON file:
//   {"mpcg_tune_cache": 1, "entries": [
//     {"arch": "gfx950", "scheme": 0, "mode": 1, "log2_m": 11, "log2_n": 11,
//      "log2_k": 11, "s_bucket": 20, "band": 20, "groups": 512, "mode3m": 1,
//      "us": 415000.0}, ...]}
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "mpcg_internal.h"

namespace mpcg {
namespace {

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;
std::string g_arch;  // the current device's architecture name, e.g. gfx950

int ceil_log2i(long long v) {
  int l = 0;
  while ((1ll << l) < v) ++l;
  return l;
}

// Value of "key": in the object text `obj` (a number, or a string for arch).
bool field(const std::string& obj, const char* key, std::string* out) {
  const std::string pat = std::string("\"") + key + "\"";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + pat.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t' || obj[p] == '\n' || obj[p] == '\r')) ++p;
  if (p < obj.size() && obj[p] == '"') {
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos) return false;
    *out = obj.substr(p + 1, q - p - 1);
    return true;
  }
  size_t q = p;
  while (q < obj.size() && (isdigit((unsigned char)obj[q]) || obj[q] == '-' || obj[q] == '+' || obj[q] == '.' ||
                            obj[q] == 'e' || obj[q] == 'E'))
    ++q;
  if (q == p) return false;
  *out = obj.substr(p, q - p);
  return true;
}

}  // namespace

bool operator<(const TuneKey& a, const TuneKey& b) {
  return std::tie(a.scheme, a.mode, a.lm, a.ln, a.lk, a.sb) < std::tie(b.scheme, b.mode, b.lm, b.ln, b.lk, b.sb);
}

TuneKey tune_key(int scheme, int mode, int m, int n, int k, int S) {
  return TuneKey{scheme, mode, ceil_log2i(m), ceil_log2i(n), ceil_log2i(k), (S + 7) / 8};
}

const char* tune_arch() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (g_arch.empty()) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      std::string a = prop.gcnArchName;
      g_arch = a.substr(0, a.find(':'));  // drop feature suffixes such as :sramecc+:xnack-
    } else {
      g_arch = "unknown";
    }
  }
  return g_arch.c_str();
}

bool tune_find(const TuneKey& key, TuneChoice* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (g_tune.empty()) return false;
  const auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void tune_put(const TuneKey& key, const TuneChoice& c) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = c;
}

int tune_count() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return (int)g_tune.size();
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
}

// Entries of `path` for this device's architecture merged into the cache;
// returns how many, or -1 if the file cannot be read or parsed.
int tune_load(const char* path) {
  const std::string arch = tune_arch();
  FILE* f = fopen(path, "rb");
  if (!f) return -1;
  std::string text;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, r);
  fclose(f);
  if (text.find("\"mpcg_tune_cache\"") == std::string::npos) return -1;
  const size_t e0 = text.find("\"entries\"");
  if (e0 == std::string::npos) return -1;
  int loaded = 0;
  size_t p = text.find('[', e0);
  if (p == std::string::npos) return -1;
  for (;;) {
    const size_t a = text.find('{', p);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) return -1;
    const std::string obj = text.substr(a, b - a + 1);
    p = b + 1;
    std::string v[11];
    static const char* keys[11] = {"arch", "scheme", "mode", "log2_m", "log2_n", "log2_k",
                                   "s_bucket", "band", "groups", "mode3m", "us"};
    bool ok = true;
    for (int i = 0; i < 11 && ok; ++i) ok = field(obj, keys[i], &v[i]);
    if (!ok) return -1;
    if (v[0] != arch) continue;
    TuneKey key{atoi(v[1].c_str()), atoi(v[2].c_str()), atoi(v[3].c_str()), atoi(v[4].c_str()),
                atoi(v[5].c_str()), atoi(v[6].c_str())};
    TuneChoice c{atoi(v[7].c_str()), atoi(v[8].c_str()), atoi(v[9].c_str()), (float)atof(v[10].c_str())};
    if (c.band != 8 && c.band != 12 && c.band != 16 && c.band != 20) return -1;
    if (c.groups < 1 || (c.mode3m != 0 && c.mode3m != 1)) return -1;
    tune_put(key, c);
    ++loaded;
  }
  return loaded;
}

int tune_save(const char* path) {
  const std::string arch = tune_arch();
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return -1;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  fprintf(f, "{\"mpcg_tune_cache\": 1, \"entries\": [");
  bool first = true;
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    const TuneChoice& c = kv.second;
    fprintf(f,
            "%s\n  {\"arch\": \"%s\", \"scheme\": %d, \"mode\": %d, \"log2_m\": %d, \"log2_n\": %d, "
            "\"log2_k\": %d, \"s_bucket\": %d, \"band\": %d, \"groups\": %d, \"mode3m\": %d, \"us\": %.1f}",
            first ? "" : ",", arch.c_str(), k.scheme, k.mode, k.lm, k.ln, k.lk, k.sb, c.band, c.groups, c.mode3m,
            c.us);
    first = false;
  }
  fprintf(f, "\n]}\n");
  const bool bad = ferror(f) != 0;
  if (fclose(f) != 0 || bad) return -1;
  if (rename(tmp.c_str(), path) != 0) return -1;
  return (int)g_tune.size();
}

}  // namespace mpcg
