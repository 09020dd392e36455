// Autotune cache of the C ABI: launch shapes the library's autotuners picked, keyed by GPU
// architecture and shape class, kept in memory behind one mutex and mirrored to a JSON file.
//
// File format (written by this library; a file that does not parse reads as empty and is
// rewritten by the next store):
//   {
//    "<key>": {"variant": 2, "pixels_per_lane": 4, "waves": 4, "us": 35.125},
//    ...
//   }
// Stores write a temporary file next to the cache and rename it over the cache, so a reader
// never sees a partial file.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "rosar_internal.hpp"

namespace {

struct Entry {
  rosar_tile tile;
  float us;
};

std::mutex g_mu;
std::string g_path;                      // empty: entries stay in memory only
std::map<std::string, Entry> g_entries;
bool g_env_read = false;

// ---------------------------------------------------------------- a parser for the format above
struct Parser {
  const char* p;
  const char* end;

  void ws() {
    while (p < end && std::isspace((unsigned char)*p)) ++p;
  }
  bool lit(char c) {
    ws();
    if (p < end && *p == c) {
      ++p;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (p >= end || *p != '"') return false;
    ++p;
    out->clear();
    while (p < end && *p != '"') {
      char c = *p++;
      if (c == '\\') {
        if (p >= end) return false;
        c = *p++;
        if (c != '"' && c != '\\' && c != '/') return false;
      }
      out->push_back(c);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool num(double* v) {
    ws();
    char* q = nullptr;
    *v = std::strtod(p, &q);
    if (q == p || q > end) return false;
    p = q;
    return true;
  }
  // {"field": number, ...}
  bool entry(Entry* e) {
    if (!lit('{')) return false;
    double variant = -1, ppl = -1, waves = -1, us = -1;
    if (lit('}')) return false;
    do {
      std::string k;
      double v = 0;
      if (!str(&k) || !lit(':') || !num(&v)) return false;
      if (k == "variant") variant = v;
      else if (k == "pixels_per_lane") ppl = v;
      else if (k == "waves") waves = v;
      else if (k == "us") us = v;
    } while (lit(','));
    if (!lit('}')) return false;
    if (variant < 0 || ppl < 0 || waves < 0 || !(us >= 0)) return false;
    e->tile = rosar_tile{(int32_t)variant, (int32_t)ppl, (int32_t)waves, 0};
    e->us = (float)us;
    return true;
  }
  bool all(std::map<std::string, Entry>* out) {
    if (!lit('{')) return false;
    if (lit('}')) return true;
    do {
      std::string k;
      Entry e{};
      if (!str(&k) || !lit(':') || !entry(&e)) return false;
      (*out)[k] = e;
    } while (lit(','));
    if (!lit('}')) return false;
    ws();
    return p == end;
  }
};

// Entries of the file at `path` (empty when missing or unparsable).  Caller holds g_mu.
std::map<std::string, Entry> read_file(const std::string& path) {
  std::map<std::string, Entry> m;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return m;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  Parser ps{text.data(), text.data() + text.size()};
  if (!ps.all(&m)) m.clear();
  return m;
}

void put_escaped(FILE* f, const std::string& s) {
  std::fputc('"', f);
  for (char c : s) {
    if (c == '"' || c == '\\') std::fputc('\\', f);
    std::fputc(c, f);
  }
  std::fputc('"', f);
}

// Writes every entry to `path` through a temporary file and a rename.  Caller holds g_mu.
bool write_file(const std::string& path, const std::map<std::string, Entry>& m) {
  const std::string tmp = path + "." + std::to_string((long)getpid()) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fputs("{\n", f);
  size_t i = 0;
  for (const auto& kv : m) {
    std::fputc(' ', f);
    put_escaped(f, kv.first);
    std::fprintf(f, ": {\"variant\": %d, \"pixels_per_lane\": %d, \"waves\": %d, \"us\": %.9g}%s\n",
                 kv.second.tile.variant, kv.second.tile.pixels_per_lane, kv.second.tile.waves, (double)kv.second.us,
                 ++i < m.size() ? "," : "");
  }
  std::fputs("}\n", f);
  const bool ok = std::fflush(f) == 0;
  std::fclose(f);
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

// First use: ROSAR_AUTOTUNE_CACHE, when set, selects the cache file.  Caller holds g_mu.
void read_env_once() {
  if (g_env_read) return;
  g_env_read = true;
  const char* v = std::getenv("ROSAR_AUTOTUNE_CACHE");
  if (v && *v) {
    g_path = v;
    g_entries = read_file(g_path);
  }
}

}  // namespace

namespace rosar {

bool tune_cache_get(const std::string& key, rosar_tile* tile, float* us) {
  std::lock_guard<std::mutex> lk(g_mu);
  read_env_once();
  const auto it = g_entries.find(key);
  if (it == g_entries.end()) return false;
  *tile = it->second.tile;
  *us = it->second.us;
  return true;
}

bool tune_cache_put(const std::string& key, const rosar_tile& tile, float us) {
  std::lock_guard<std::mutex> lk(g_mu);
  read_env_once();
  g_entries[key] = Entry{tile, us};
  if (g_path.empty()) return true;
  // merge with what other processes wrote since the file was read
  std::map<std::string, Entry> m = read_file(g_path);
  m[key] = Entry{tile, us};
  g_entries = m;
  return write_file(g_path, m);
}

std::string tune_arch() {
  int dev = -1;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');   // drop the target features
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace rosar

extern "C" {

rosar_status rosar_autotune(const char* cache_path) {
  rosar::clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_read = true;   // an explicit choice overrides the environment
  g_path = cache_path ? cache_path : "";
  g_entries = g_path.empty() ? std::map<std::string, Entry>{} : read_file(g_path);
  return ROSAR_OK;
}

rosar_status rosar_autotune_lookup(const char* key, rosar_tile* tile, float* us, int32_t* found) {
  rosar::clear_error();
  if (!key || !tile || !us || !found) return rosar::set_error(ROSAR_ERR_INVALID_ARG, "key, tile, us or found is NULL");
  *found = rosar::tune_cache_get(key, tile, us) ? 1 : 0;
  return ROSAR_OK;
}

rosar_status rosar_autotune_store(const char* key, const rosar_tile* tile, float us) {
  rosar::clear_error();
  if (!key || !*key || !tile) return rosar::set_error(ROSAR_ERR_INVALID_ARG, "key empty or NULL, or tile NULL");
  if (!(us >= 0.f)) return rosar::set_error(ROSAR_ERR_INVALID_ARG, "us must be >= 0");
  if (!rosar::tune_cache_put(key, *tile, us))
    return rosar::set_error(ROSAR_ERR_INVALID_ARG, "cannot write the autotune cache file");
  return ROSAR_OK;
}

}  // extern "C"
