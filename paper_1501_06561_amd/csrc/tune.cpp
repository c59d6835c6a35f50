// Launch-shape tuner: choice table, cache file and the C ABI that controls
// them (see fdsk_tune.hpp and include/fdsketch.h).
#include "fdsk_tune.hpp"

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "fdsketch.h"

namespace fdsk {
namespace {

struct Table {
  std::mutex mu;
  bool init = false;
  int mode = TUNE_ON;
  std::string path;                    // cache file ("" = none)
  std::map<std::string, int> value;    // key -> choice
  std::map<std::string, std::string> note;   // key -> timings of the candidates
  std::string last_error;
};

Table& table() {
  static Table t;
  return t;
}

std::string default_path() {
  if (const char* p = std::getenv("FDSK_TUNE_CACHE")) return p;
  std::string dir;
  if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x)
    dir = x;
  else if (const char* h = std::getenv("HOME"); h && *h)
    dir = std::string(h) + "/.cache";
  else
    return "";
  return dir + "/fdsketch/tune.tsv";
}

// Merge "key<TAB>value[<TAB>note]" lines of path into the table (entries
// already present are replaced).  Returns false when the file cannot be read.
bool load_locked(Table& t, const std::string& path) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    const size_t a = line.find('\t');
    if (a == std::string::npos || a == 0) continue;
    const size_t b = line.find('\t', a + 1);
    const std::string v = line.substr(a + 1, b == std::string::npos ? std::string::npos : b - a - 1);
    char* end = nullptr;
    const long x = std::strtol(v.c_str(), &end, 10);
    if (end == v.c_str() || *end != '\0') continue;
    const std::string key = line.substr(0, a);
    t.value[key] = static_cast<int>(x);
    if (b != std::string::npos) t.note[key] = line.substr(b + 1);
  }
  return true;
}

void mkdirs(const std::string& file) {
  for (size_t p = file.find('/', 1); p != std::string::npos; p = file.find('/', p + 1))
    ::mkdir(file.substr(0, p).c_str(), 0755);
}

// Write the whole table to path (through a temporary file and a rename).
bool save_locked(Table& t, const std::string& path) {
  if (path.empty()) return false;
  mkdirs(path);
  const std::string tmp = path + ".tmp." + std::to_string(static_cast<long>(::getpid()));
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) {
      t.last_error = "cannot write " + tmp + ": " + std::strerror(errno);
      return false;
    }
    out << "# fdsketch launch-shape cache: key<TAB>choice<TAB>candidate:microseconds ...\n";
    for (const auto& kv : t.value) {
      out << kv.first << '\t' << kv.second;
      auto it = t.note.find(kv.first);
      if (it != t.note.end() && !it->second.empty()) out << '\t' << it->second;
      out << '\n';
    }
    if (!out) {
      t.last_error = "writing " + tmp + " failed";
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    t.last_error = "cannot rename " + tmp + ": " + std::strerror(errno);
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

// First use: mode from FDSK_TUNE, cache path, and the cache's entries.
void ensure_init_locked(Table& t) {
  if (t.init) return;
  t.init = true;
  if (const char* m = std::getenv("FDSK_TUNE")) {
    if (!std::strcmp(m, "0") || !std::strcmp(m, "off")) t.mode = TUNE_OFF;
    else if (!std::strcmp(m, "refresh") || !std::strcmp(m, "2")) t.mode = TUNE_REFRESH;
    else t.mode = TUNE_ON;
  }
  t.path = default_path();
  if (!t.path.empty()) load_locked(t, t.path);
}

}  // namespace

int tune_mode() {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  return t.mode;
}

std::string tune_device_tag() {
  int dev = 0;
  hipDeviceProp_t p{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string arch = p.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch = arch.substr(0, c);
  return arch + "/" + std::to_string(p.multiProcessorCount);
}

int tune_bucket(int x) {
  int b = 1;
  while (b < x) b <<= 1;
  return b;
}

int tune_pick(const std::string& key, const std::vector<int>& candidates, int dflt, hipStream_t s,
              const std::function<hipError_t(int)>& launch, int reps) {
  Table& t = table();
  {
    std::lock_guard<std::mutex> g(t.mu);
    ensure_init_locked(t);
    if (t.mode == TUNE_OFF) return dflt;
    if (t.mode == TUNE_ON) {
      auto it = t.value.find(key);
      if (it != t.value.end() &&
          std::find(candidates.begin(), candidates.end(), it->second) != candidates.end())
        return it->second;
    }
  }
  if (candidates.size() <= 1) return candidates.empty() ? dflt : candidates[0];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return dflt;
  }
  std::vector<std::pair<int, float>> timed;
  for (int c : candidates) {
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = launch(c);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(c);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) {
      timed.push_back({c, 1000.f * ms / reps});
    } else {
      (void)hipGetLastError();   // a refused launch shape is skipped
      (void)hipStreamSynchronize(s);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (timed.empty()) return dflt;
  float t_def = -1.f;
  for (auto& ct : timed)
    if (ct.first == dflt) t_def = ct.second;
  auto best = std::min_element(timed.begin(), timed.end(),
                               [](const auto& a, const auto& b) { return a.second < b.second; });
  int choice = best->first;
  if (t_def >= 0.f && best->second > 0.97f * t_def) choice = dflt;
  std::ostringstream note;
  for (size_t i = 0; i < timed.size(); ++i)
    note << (i ? " " : "") << timed[i].first << ':' << static_cast<int>(timed[i].second * 10.f + 0.5f) / 10.0;
  std::lock_guard<std::mutex> g(t.mu);
  t.value[key] = choice;
  t.note[key] = note.str();
  if (!t.path.empty()) save_locked(t, t.path);
  return choice;
}

}  // namespace fdsk

using namespace fdsk;

extern "C" {

int fdsk_tune_set_mode(int32_t mode) {
  if (mode < TUNE_OFF || mode > TUNE_REFRESH) return FDSK_EINVAL;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  t.mode = mode;
  return 0;
}

int fdsk_tune_get_mode(void) { return tune_mode(); }

int fdsk_tune_lookup(const char* key, int32_t* value) {
  if (!key || !value) return FDSK_EINVAL;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  auto it = t.value.find(key);
  if (it == t.value.end()) return 1;
  *value = it->second;
  return 0;
}

int fdsk_tune_set(const char* key, int32_t value) {
  if (!key || !*key || std::strchr(key, '\t') || std::strchr(key, '\n')) return FDSK_EINVAL;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  t.value[key] = value;
  t.note[key] = "set";
  return 0;
}

int fdsk_tune_clear(void) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  t.value.clear();
  t.note.clear();
  return 0;
}

int fdsk_tune_set_path(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  t.path = path ? path : "";
  return 0;
}

const char* fdsk_tune_path(void) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  return t.path.c_str();
}

int fdsk_tune_load(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  const std::string p = path ? std::string(path) : t.path;
  if (p.empty() || !load_locked(t, p)) {
    t.last_error = "cannot read " + p;
    return FDSK_EINVAL;
  }
  return 0;
}

int fdsk_tune_save(const char* path) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  const std::string p = path ? std::string(path) : t.path;
  if (p.empty()) {
    t.last_error = "no cache path";
    return FDSK_EINVAL;
  }
  return save_locked(t, p) ? 0 : FDSK_EDEVICE;
}

int32_t fdsk_tune_dump(char* buf, int64_t cap) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  ensure_init_locked(t);
  std::string s;
  for (const auto& kv : t.value) {
    s += kv.first + '\t' + std::to_string(kv.second);
    auto it = t.note.find(kv.first);
    if (it != t.note.end() && !it->second.empty()) s += '\t' + it->second;
    s += '\n';
  }
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(s.size(), static_cast<size_t>(cap - 1));
    std::memcpy(buf, s.data(), n);
    buf[n] = '\0';
  }
  return static_cast<int32_t>(s.size());
}

const char* fdsk_tune_last_error(void) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  return t.last_error.c_str();
}

}  // extern "C"
