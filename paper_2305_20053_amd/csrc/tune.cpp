// Persisted autotuning choices: a text file of "key value" lines, loaded
// once per process and appended to as choices are made.  The library times
// the candidate launch shapes of a kernel at its first use for a given size
// and records the fastest here, so later processes on the same device skip
// the timing.
#include "tune.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include <sys/stat.h>

namespace saa_tune {
namespace {

std::mutex mu;
bool loaded = false;
std::map<std::string, int> table;

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t p{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  char buf[96];
  std::snprintf(buf, sizeof(buf), "%s:cu%d", p.gcnArchName, p.multiProcessorCount);
  for (char* c = buf; *c; ++c)
    if (*c == ' ') *c = '_';
  return buf;
}

void load_locked() {
  if (loaded) return;
  loaded = true;
  const std::string f = path();
  if (f.empty()) return;
  FILE* fp = std::fopen(f.c_str(), "r");
  if (!fp) return;
  char key[512];
  int value = 0;
  while (std::fscanf(fp, "%511s %d", key, &value) == 2) table[key] = value;
  std::fclose(fp);
}

}  // namespace

std::string path() {
  const char* env = std::getenv("SAA_TUNE_CACHE");
  if (env && *env) return std::strcmp(env, "off") == 0 ? std::string() : std::string(env);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/saa_tune.txt";
}

int lookup(const std::string& key) {
  const std::string k = device_tag() + "/" + key;
  std::lock_guard<std::mutex> lock(mu);
  load_locked();
  auto it = table.find(k);
  return it == table.end() ? -1 : it->second;
}

void store(const std::string& key, int value) {
  const std::string k = device_tag() + "/" + key;
  std::lock_guard<std::mutex> lock(mu);
  load_locked();
  table[k] = value;
  const std::string f = path();
  if (f.empty()) return;
  const size_t slash = f.rfind('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(f.substr(0, slash).c_str(), 0755);   // one level
  FILE* fp = std::fopen(f.c_str(), "a");
  if (!fp) return;   // not persisted (read-only location): the choice stays in memory
  std::fprintf(fp, "%s %d\n", k.c_str(), value);
  std::fclose(fp);
}

}  // namespace saa_tune
