// Persistent autotuning choices.  The file named by PRUNE_AUTOTUNE_CACHE
// holds one JSON object per line,
//   {"key": "<shape class>", "choice": "<kernel variant name>", "ms": <time>}
// read once per process on the first lookup and appended to after every new
// tuning run; a later line for the same key overrides an earlier one.  Keys
// name the kernel family, the device architecture and the shape class, so a
// file may be shared between devices and library versions: a choice whose
// name is no longer a variant is ignored by the caller.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "prune.h"
#include "runtime_kernels.h"

namespace prune {

namespace {

std::mutex g_mu;
bool g_loaded = false;
uint32_t g_stores = 0, g_hits = 0;   // tuning runs recorded, choices found in the file
std::map<std::string, std::string> g_file;   // key -> choice, as read from the file

// The string value of "field": "..." in one line, or empty.
std::string json_field(const std::string &line, const char *field) {
  const std::string tag = std::string("\"") + field + "\"";
  size_t p = line.find(tag);
  if (p == std::string::npos) return {};
  p = line.find(':', p + tag.size());
  if (p == std::string::npos) return {};
  p = line.find('"', p);
  if (p == std::string::npos) return {};
  const size_t e = line.find('"', p + 1);
  if (e == std::string::npos) return {};
  return line.substr(p + 1, e - p - 1);
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char *path = getenv("PRUNE_AUTOTUNE_CACHE");
  if (!path || !path[0]) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    const std::string line(buf);
    const std::string k = json_field(line, "key"), c = json_field(line, "choice");
    if (!k.empty() && !c.empty()) g_file[k] = c;
  }
  fclose(f);
}

}  // namespace

std::string tune_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

bool tune_cache_lookup(const std::string &key, std::string *choice) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  auto it = g_file.find(key);
  if (it == g_file.end()) return false;
  *choice = it->second;
  ++g_hits;
  return true;
}

void tune_cache_store(const std::string &key, const char *choice, double ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  g_file[key] = choice;
  ++g_stores;
  const char *path = getenv("PRUNE_AUTOTUNE_CACHE");
  if (!path || !path[0]) return;
  if (FILE *f = fopen(path, "a")) {
    fprintf(f, "{\"key\": \"%s\", \"choice\": \"%s\", \"ms\": %.5f}\n", key.c_str(), choice, ms);
    fclose(f);
  }
}

void tune_cache_counts(uint32_t *runs, uint32_t *hits) {
  std::lock_guard<std::mutex> lk(g_mu);
  *runs = g_stores;
  *hits = g_hits;
}

}  // namespace prune

extern "C" prune_status prune_autotune_counts(uint32_t *tuning_runs, uint32_t *cache_hits) {
  if (!tuning_runs || !cache_hits) return PRUNE_E_ARG;
  prune::tune_cache_counts(tuning_runs, cache_hits);
  return PRUNE_OK;
}
