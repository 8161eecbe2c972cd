// Persistent autotune cache: tile-class tables of the batched kernel stored
// as JSON, one table per line, keyed by device architecture, CU count,
// element type and library version, so that a process does not re-time the
// 216 shape buckets a previous process already timed on the same part.
//
//   {"format": "mg-autotune-1", "tables": [
//   {"arch": "gfx950:sramecc+:xnack-", "cus": 256, "dtype": "f64", "lib": 10100, "classes": [...]},
//   ...
//   ]}
//
// Entries with another key are kept when the file is rewritten; a line that
// does not parse as an entry is dropped.  The file is replaced atomically
// (written to a temporary name, then renamed).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "grouped.h"

namespace mg {

int64_t now_ns();  // the server's steady clock

namespace {

struct CacheEntry {
  std::string arch;
  long long cus = 0, lib = 0;
  std::string dtype;
  std::vector<int> classes;
};

const char *dtype_name(int dtype) { return dtype == MG_F64 ? "f64" : "f32"; }

// Value of "key": as a string (quoted) or a raw token; false if absent.
bool field(const std::string &line, const char *key, std::string *out) {
  const std::string pat = std::string("\"") + key + "\":";
  size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  p += pat.size();
  while (p < line.size() && line[p] == ' ') ++p;
  if (p < line.size() && line[p] == '"') {
    const size_t e = line.find('"', p + 1);
    if (e == std::string::npos) return false;
    *out = line.substr(p + 1, e - p - 1);
    return true;
  }
  size_t e = p;
  while (e < line.size() && line[e] != ',' && line[e] != '}') ++e;
  *out = line.substr(p, e - p);
  return !out->empty();
}

bool parse_entry(const std::string &line, CacheEntry *e) {
  std::string v;
  if (!field(line, "arch", &e->arch) || !field(line, "dtype", &e->dtype)) return false;
  if (!field(line, "cus", &v)) return false;
  e->cus = std::atoll(v.c_str());
  if (!field(line, "lib", &v)) return false;
  e->lib = std::atoll(v.c_str());
  const size_t b = line.find("\"classes\":");
  if (b == std::string::npos) return false;
  const size_t lo = line.find('[', b), hi = line.find(']', b);
  if (lo == std::string::npos || hi == std::string::npos || hi < lo) return false;
  std::stringstream ss(line.substr(lo + 1, hi - lo - 1));
  std::string tok;
  e->classes.clear();
  while (std::getline(ss, tok, ',')) {
    char *end = nullptr;
    const long c = std::strtol(tok.c_str(), &end, 10);
    if (end == tok.c_str() || c < 0 || c >= kNumGroupedClasses) return false;
    e->classes.push_back((int)c);
  }
  return (int)e->classes.size() == MG_TUNE_BUCKETS;
}

std::vector<CacheEntry> read_cache(const char *path) {
  std::vector<CacheEntry> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    CacheEntry e;
    if (parse_entry(line, &e)) out.push_back(e);
  }
  return out;
}

int device_key(std::string *arch, long long *cus) {
  int dev = 0;
  MG_HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  MG_HIP_TRY(hipGetDeviceProperties(&prop, dev));
  *arch = prop.gcnArchName;
  *cus = prop.multiProcessorCount;
  return MG_OK;
}

bool same_key(const CacheEntry &e, const std::string &arch, long long cus, int dtype) {
  return e.arch == arch && e.cus == cus && e.dtype == dtype_name(dtype) && e.lib == mg_version();
}

int write_cache(const char *path, const std::vector<CacheEntry> &entries) {
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)now_ns());
  {
    std::ofstream f(tmp);
    if (!f) {
      set_error("cannot write autotune cache %s", tmp.c_str());
      return MG_ERR_INVALID_ARG;
    }
    f << "{\"format\": \"mg-autotune-1\", \"tables\": [\n";
    for (size_t i = 0; i < entries.size(); ++i) {
      const CacheEntry &e = entries[i];
      f << "{\"arch\": \"" << e.arch << "\", \"cus\": " << e.cus << ", \"dtype\": \"" << e.dtype
        << "\", \"lib\": " << e.lib << ", \"classes\": [";
      for (size_t j = 0; j < e.classes.size(); ++j) f << (j ? "," : "") << e.classes[j];
      f << "]}" << (i + 1 < entries.size() ? "," : "") << "\n";
    }
    f << "]}\n";
    if (!f) {
      set_error("cannot write autotune cache %s", tmp.c_str());
      return MG_ERR_INVALID_ARG;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    set_error("cannot replace autotune cache %s", path);
    return MG_ERR_INVALID_ARG;
  }
  return MG_OK;
}

}  // namespace

int autotune_cached(int dtype, int reps, const char *path, hipStream_t s, mg_tune_table *out,
                    int *from_cache) {
  if (from_cache) *from_cache = 0;
  if (path == nullptr || path[0] == '\0') return autotune(dtype, reps, s, out);
  std::string arch;
  long long cus = 0;
  int rc = device_key(&arch, &cus);
  if (rc != MG_OK) return rc;
  std::vector<CacheEntry> entries = read_cache(path);
  for (const CacheEntry &e : entries)
    if (same_key(e, arch, cus, dtype)) {
      out->dtype = dtype;
      for (int b = 0; b < MG_TUNE_BUCKETS; ++b) out->cls[b] = e.classes[(size_t)b];
      if (from_cache) *from_cache = 1;
      return MG_OK;
    }
  rc = autotune(dtype, reps, s, out);
  if (rc != MG_OK) return rc;
  CacheEntry mine;
  mine.arch = arch;
  mine.cus = cus;
  mine.dtype = dtype_name(dtype);
  mine.lib = mg_version();
  mine.classes.assign(out->cls, out->cls + MG_TUNE_BUCKETS);
  std::vector<CacheEntry> keep;
  for (const CacheEntry &e : entries)
    if (!same_key(e, arch, cus, dtype)) keep.push_back(e);
  keep.push_back(mine);
  return write_cache(path, keep);
}

}  // namespace mg
