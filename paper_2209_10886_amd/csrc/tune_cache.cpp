// Persistent cache of autotuned launch choices (host code only).
//
// The file is one JSON object
//   {"version": 1, "entries": {"<key>": {"variant": v, "us": [t0, t1, ...]}, ...}}
// where the key names the kernel family, the precision, the problem shape and the batch class
// the choice was timed on, "variant" is the chosen launch variant and "us" the measured
// microseconds of every candidate (0 for one that was not timed).  The cache is read once per
// process (lazily, on the first lookup), and after every new decision it is merged with what is on
// disk (other processes may have added entries) and rewritten atomically: a temporary file in the
// same directory, then rename.
//
// Location: the environment variable HBJ_TUNE_CACHE if it is set ("" or "off": no file, decisions
// live in this process only), else $XDG_CACHE_HOME/hbj/tune.json, else $HOME/.cache/hbj/tune.json.
// hbj_tune_cache_set_path overrides all of these.
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hbj.h"
#include "hbj_internal.h"

namespace {

struct TuneEntry {
  int variant = 0;
  std::vector<float> us;
};

struct TuneCache {
  std::mutex mu;
  bool path_set = false;  // path resolved (from the environment or set explicitly)
  bool loaded = false;
  std::string path;       // empty: no file
  std::map<std::string, TuneEntry> entries;
};

TuneCache& cache() {
  static TuneCache c;
  return c;
}

std::string default_path() {
  const char* env = std::getenv("HBJ_TUNE_CACHE");
  if (env) {
    if (!*env || std::strcmp(env, "off") == 0) return std::string();
    return std::string(env);
  }
  const char* xdg = std::getenv("XDG_CACHE_HOME");
  if (xdg && *xdg) return std::string(xdg) + "/hbj/tune.json";
  const char* home = std::getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/hbj/tune.json";
  return std::string();
}

// keys are plain identifiers: letters, digits and _ . - x | (no quoting needed in JSON)
bool key_ok(const char* k) {
  if (!k || !*k || std::strlen(k) > 200) return false;
  for (const char* p = k; *p; ++p) {
    const char ch = *p;
    const bool ok = (ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') || ch == '_' ||
                    ch == '.' || ch == '-' || ch == '|' || ch == ':';
    if (!ok) return false;
  }
  return true;
}

// ---- a small reader for the subset of JSON the writer produces (objects, arrays, strings
// without escapes, numbers); anything else makes the whole file count as empty
struct Reader {
  const char* p;
  const char* end;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(char ch) {
    ws();
    if (p < end && *p == ch) {
      ++p;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    ws();
    if (p >= end || *p != '"') return false;
    ++p;
    const char* b = p;
    while (p < end && *p != '"') {
      if (*p == '\\') return false;
      ++p;
    }
    if (p >= end) return false;
    out.assign(b, p - b);
    ++p;
    return true;
  }
  bool num(double& v) {
    ws();
    char* e = nullptr;
    errno = 0;
    v = std::strtod(p, &e);
    if (e == p || e > end || errno == ERANGE) return false;
    p = e;
    return true;
  }
  bool entry(TuneEntry& t) {
    if (!lit('{')) return false;
    bool have_v = false;
    if (lit('}')) return false;
    do {
      std::string k;
      if (!str(k) || !lit(':')) return false;
      if (k == "variant") {
        double v;
        if (!num(v) || v != (double)(int)v) return false;
        t.variant = (int)v;
        have_v = true;
      } else if (k == "us") {
        if (!lit('[')) return false;
        if (!lit(']')) {
          do {
            double v;
            if (!num(v)) return false;
            t.us.push_back((float)v);
          } while (lit(','));
          if (!lit(']')) return false;
        }
      } else {
        return false;
      }
    } while (lit(','));
    return lit('}') && have_v;
  }
  bool file(std::map<std::string, TuneEntry>& out) {
    if (!lit('{')) return false;
    bool have_entries = false;
    if (!lit('}')) {
      do {
        std::string k;
        if (!str(k) || !lit(':')) return false;
        if (k == "version") {
          double v;
          if (!num(v) || v != 1.0) return false;
        } else if (k == "entries") {
          if (!lit('{')) return false;
          if (!lit('}')) {
            do {
              std::string key;
              TuneEntry t;
              if (!str(key) || !key_ok(key.c_str()) || !lit(':') || !entry(t)) return false;
              out[key] = t;
            } while (lit(','));
            if (!lit('}')) return false;
          }
          have_entries = true;
        } else {
          return false;
        }
      } while (lit(','));
      if (!lit('}')) return false;
    }
    ws();
    return have_entries && p == end;
  }
};

bool read_file(const std::string& path, std::map<std::string, TuneEntry>& out) {
  out.clear();
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, n);
    if (text.size() > ((size_t)16 << 20)) break;  // not ours
  }
  std::fclose(f);
  Reader r{text.data(), text.data() + text.size()};
  std::map<std::string, TuneEntry> tmp;
  if (!r.file(tmp)) return false;
  out.swap(tmp);
  return true;
}

bool make_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i) {
    if (path[i] != '/') continue;
    const std::string d = path.substr(0, i);
    if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

bool write_file(const std::string& path, const std::map<std::string, TuneEntry>& ents) {
  if (!make_dirs(path)) return false;
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{\"version\": 1, \"entries\": {");
  bool first = true;
  for (const auto& kv : ents) {
    std::fprintf(f, "%s\n  \"%s\": {\"variant\": %d, \"us\": [", first ? "" : ",", kv.first.c_str(), kv.second.variant);
    for (size_t i = 0; i < kv.second.us.size(); ++i)
      std::fprintf(f, "%s%.3f", i ? ", " : "", (double)kv.second.us[i]);
    std::fprintf(f, "]}");
    first = false;
  }
  std::fprintf(f, "\n}}\n");
  const bool ok = std::fflush(f) == 0;
  std::fclose(f);
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

void ensure_loaded(TuneCache& c) {
  if (!c.path_set) {
    c.path = default_path();
    c.path_set = true;
  }
  if (c.loaded) return;
  c.loaded = true;
  if (!c.path.empty()) read_file(c.path, c.entries);
}

}  // namespace

bool tune_cache_get(const std::string& key, int* variant) {
  TuneCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  ensure_loaded(c);
  auto it = c.entries.find(key);
  if (it == c.entries.end()) return false;
  *variant = it->second.variant;
  return true;
}

bool tune_cache_put(const std::string& key, int variant, const float* us, int n) {
  if (!key_ok(key.c_str()) || n < 0 || n > 64) return false;
  TuneCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  ensure_loaded(c);
  TuneEntry t;
  t.variant = variant;
  if (us) t.us.assign(us, us + n);
  c.entries[key] = t;
  if (c.path.empty()) return true;
  // merge with what other processes wrote since this one read the file (this process wins)
  std::map<std::string, TuneEntry> disk;
  read_file(c.path, disk);
  for (const auto& kv : c.entries) disk[kv.first] = kv.second;
  c.entries = disk;
  return write_file(c.path, c.entries);
}

extern "C" {

const char* hbj_tune_cache_path(void) {
  TuneCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (!c.path_set) {
    c.path = default_path();
    c.path_set = true;
  }
  static thread_local std::string out;
  out = c.path;
  return out.c_str();
}

int hbj_tune_cache_set_path(const char* path) {
  TuneCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.path = path ? std::string(path) : default_path();
  c.path_set = true;
  c.loaded = false;
  c.entries.clear();
  ensure_loaded(c);
  return HBJ_OK;
}

int hbj_tune_cache_lookup(const char* key, int32_t* variant) {
  if (!key || !variant) return HBJ_EINVAL;
  int v = 0;
  if (!tune_cache_get(key, &v)) return 0;
  *variant = v;
  return 1;
}

int hbj_tune_cache_store(const char* key, int32_t variant, const float* us, int32_t n) {
  if (!key || !key_ok(key) || n < 0 || n > 64 || (n > 0 && !us)) return HBJ_EINVAL;
  return tune_cache_put(key, variant, us, n) ? HBJ_OK : HBJ_EIO;
}

int32_t hbj_tune_cache_size(void) {
  TuneCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  ensure_loaded(c);
  return (int32_t)c.entries.size();
}

}  // extern "C"
