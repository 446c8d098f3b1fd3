// Persistent store of the CG launch-shape autotuner.
//
// The tuner (block_cg_multi in cg.hip) times candidate launch shapes of the
// block CG on the caller's own problem the first time a problem class is
// met, and keeps the fastest here, keyed by the problem class, so that later
// calls -- in this process or another one -- start from it.  The store is a
// small JSON object, one entry per line:
//   {
//   "gfx950|ni16|ns1|b1|n19|r12|lr1": {"spmm_blocks": 32768, "update_blocks": 768, "union_spmm": 1, "fw_mfma": 1, "ms_per_iter": 1.14, "default_ms_per_iter": 1.15},
//   ...
//   }
// Reading is tolerant: lines that do not parse are skipped, and a missing
// or unreadable file is an empty store.  Writing replaces the file
// atomically (temporary file + rename), so concurrent writers lose updates
// at worst, never the file.
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

std::mutex g_tune_mu;   // serialises store access inside one process
// entries stored by this process, by (path, key): kept also when the file
// cannot be written, so one process tunes each problem class once
std::map<std::pair<std::string, std::string>, TuneChoice> g_mem;

bool parse_number(const std::string& line, const char* name, double* out) {
  const std::string pat = std::string("\"") + name + "\"";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  size_t q = line.find(':', p + pat.size());
  if (q == std::string::npos) return false;
  ++q;
  while (q < line.size() && line[q] == ' ') ++q;
  const char* s = line.c_str() + q;
  char* end = nullptr;
  errno = 0;
  const double v = std::strtod(s, &end);
  if (end == s || errno != 0 || !std::isfinite(v)) return false;
  *out = v;
  return true;
}

// key -> entry line (without a trailing comma)
std::map<std::string, std::string> read_store(const std::string& path) {
  std::map<std::string, std::string> m;
  std::ifstream f(path);
  if (!f) return m;
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    if (b == std::string::npos) continue;
    const size_t brace = line.find('{', b);
    const size_t close = line.rfind('}');
    if (brace == std::string::npos || close == std::string::npos || close < brace) continue;
    TuneChoice t;
    if (!parse_entry(line, &t)) continue;
    m[line.substr(a + 1, b - a - 1)] = format_entry(line.substr(a + 1, b - a - 1), t);
  }
  return m;
}

void mkdirs_for(const std::string& path) {
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1)) {
    const std::string d = path.substr(0, p);
    if (::mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return;
  }
}

}  // namespace

bool parse_entry(const std::string& line, TuneChoice* t) {
  double v[4];
  static const char* names[4] = {"spmm_blocks", "update_blocks", "union_spmm", "fw_mfma"};
  for (int k = 0; k < 4; ++k)
    if (!parse_number(line, names[k], &v[k]) || v[k] != std::floor(v[k])) return false;
  if (v[0] < 8 || v[0] > 65535 || std::fmod(v[0], 8.0) != 0.0) return false;
  if (v[1] < 1 || v[1] > 65535) return false;
  if (v[2] < -1 || v[2] > 1 || v[3] < -1 || v[3] > 1) return false;
  t->spmm_blocks = (int)v[0];
  t->update_blocks = (int)v[1];
  t->union_spmm = (int)v[2];
  t->fw_mfma = (int)v[3];
  double ms = 0.0, dms = 0.0;
  t->ms_per_iter = parse_number(line, "ms_per_iter", &ms) ? ms : 0.0;
  t->default_ms_per_iter = parse_number(line, "default_ms_per_iter", &dms) ? dms : 0.0;
  return true;
}

std::string format_entry(const std::string& key, const TuneChoice& t) {
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "\"%s\": {\"spmm_blocks\": %d, \"update_blocks\": %d, \"union_spmm\": %d, \"fw_mfma\": %d, "
                "\"ms_per_iter\": %.6g, \"default_ms_per_iter\": %.6g}",
                key.c_str(), t.spmm_blocks, t.update_blocks, t.union_spmm, t.fw_mfma, t.ms_per_iter,
                t.default_ms_per_iter);
  return buf;
}

std::string tune_cache_path() {
  const char* p = std::getenv("SDGP_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/sdgp/autotune.json";
  return std::string();
}

bool tune_cache_get(const std::string& path, const std::string& key, TuneChoice* out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  const auto mi = g_mem.find(std::make_pair(path, key));
  if (mi != g_mem.end()) {
    *out = mi->second;
    return true;
  }
  if (path.empty()) return false;
  const auto m = read_store(path);
  const auto it = m.find(key);
  if (it == m.end()) return false;
  return parse_entry(it->second, out);
}

bool tune_cache_put(const std::string& path, const std::string& key, const TuneChoice& t) {
  if (key.empty() || key.find('"') != std::string::npos || key.find('\n') != std::string::npos) return false;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_mem[std::make_pair(path, key)] = t;
  if (path.empty()) return false;
  auto m = read_store(path);
  m[key] = format_entry(key, t);
  mkdirs_for(path);
  const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (const auto& kv : m) f << kv.second << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) {
      f.close();
      std::remove(tmp.c_str());
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace sdgp

using namespace sdgp;

extern "C" {

sdgp_status sdgp_tune_cache_get(const char* path, const char* key, int64_t* values) {
  if (!key || !values) return SDGP_ERR_INVALID_ARG;
  TuneChoice t;
  const std::string p = path ? std::string(path) : tune_cache_path();
  if (!tune_cache_get(p, key, &t)) return SDGP_ERR_INVALID_ARG;
  values[0] = t.spmm_blocks;
  values[1] = t.update_blocks;
  values[2] = t.union_spmm;
  values[3] = t.fw_mfma;
  return SDGP_OK;
}

sdgp_status sdgp_tune_cache_put(const char* path, const char* key, const int64_t* values) {
  if (!key || !values) return SDGP_ERR_INVALID_ARG;
  TuneChoice t;
  t.spmm_blocks = (int)values[0];
  t.update_blocks = (int)values[1];
  t.union_spmm = (int)values[2];
  t.fw_mfma = (int)values[3];
  // the same validity rules as for entries read back
  if (!parse_entry(format_entry(key, t), &t)) return SDGP_ERR_INVALID_ARG;
  const std::string p = path ? std::string(path) : tune_cache_path();
  return tune_cache_put(p, key, t) ? SDGP_OK : SDGP_ERR_INVALID_ARG;
}

}  // extern "C"
