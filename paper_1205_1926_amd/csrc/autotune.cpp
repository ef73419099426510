// Autotuner cache: one JSON object per line,
//   {"key": "...", "tile": 32, "natural": 0, "threads": 256, "ms": 1.768}
// Lines that do not parse are kept as they are and ignored.
#include "autotune.h"

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>

namespace tfeti {

namespace {

uint64_t fnv1a(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xffu;
    h *= 0x100000001b3ull;
  }
  return h;
}

// Value of "name": in a line, as text up to the next ',' or '}' (quotes removed).
bool field(const std::string& line, const std::string& name, std::string* out) {
  const std::string tag = "\"" + name + "\":";
  size_t p = line.find(tag);
  if (p == std::string::npos) return false;
  p += tag.size();
  while (p < line.size() && line[p] == ' ') ++p;
  if (p < line.size() && line[p] == '"') {
    size_t e = line.find('"', p + 1);
    if (e == std::string::npos) return false;
    *out = line.substr(p + 1, e - p - 1);
    return true;
  }
  size_t e = line.find_first_of(",}", p);
  if (e == std::string::npos) return false;
  *out = line.substr(p, e - p);
  return true;
}

bool parse(const std::string& line, std::string* key, TuneChoice* c) {
  std::string k, t, n, m, w;
  if (!field(line, "key", &k) || !field(line, "tile", &t) || !field(line, "natural", &n) || !field(line, "ms", &m) ||
      !field(line, "threads", &w))
    return false;
  try {
    c->tile = std::stoi(t);
    c->natural = std::stoi(n);
    c->threads = std::stoi(w);
    c->ms = std::stod(m);
  } catch (...) {
    return false;
  }
  if (c->tile != 16 && c->tile != 32 && c->tile != 64) return false;
  if (c->natural != 0 && c->natural != 1) return false;
  if (c->threads != 256 && c->threads != 512 && c->threads != 1024) return false;
  *key = k;
  return true;
}

}  // namespace

std::string tune_key(const std::string& arch, int precision, const std::vector<int32_t>& ndofs) {
  std::map<int32_t, int64_t> hist;
  for (int32_t n : ndofs) hist[n]++;
  uint64_t h = 0xcbf29ce484222325ull;
  for (const auto& kv : hist) {
    h = fnv1a(h, (uint64_t)(uint32_t)kv.first);
    h = fnv1a(h, (uint64_t)kv.second);
  }
  char buf[64];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  std::string a = arch.substr(0, arch.find(':'));  // drop target features
  return a + "|" + (precision == 0 ? "fp64" : "fp32") + "|n=" + std::to_string(ndofs.size()) + "|h=" + buf;
}

bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice* out) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line, k;
  TuneChoice c;
  bool found = false;
  while (std::getline(f, line))
    if (parse(line, &k, &c) && k == key) {
      *out = c;
      found = true;
    }
  return found;
}

bool tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line, k;
    TuneChoice old;
    while (f && std::getline(f, line)) {
      if (parse(line, &k, &old) && k == key) continue;
      if (!line.empty()) keep.push_back(line);
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf), "{\"key\": \"%s\", \"tile\": %d, \"natural\": %d, \"threads\": %d, \"ms\": %.6f}",
                key.c_str(), c.tile, c.natural, c.threads, c.ms);
  keep.push_back(buf);
  const std::string tmp = path + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return false;
    for (const auto& l : keep) o << l << "\n";
    if (!o) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace tfeti
