// JSON cache of the autotuner (reader/writer for the flat format of tune.hpp).
#include "tune.hpp"

#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace fockmi {

namespace {

struct Reader {
  const std::string& s;
  size_t i = 0;
  explicit Reader(const std::string& str) : s(str) {}
  void ws() {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double* out) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    *out = std::strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};

}  // namespace

bool TuneCache::load(const std::string& path) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Reader r(text);
  std::map<std::string, TuneEntry> parsed;
  if (!r.eat('{')) return false;
  if (r.eat('}')) {
    entries_ = parsed;
    return true;
  }
  for (;;) {
    std::string key;
    if (!r.str(&key) || !r.eat(':') || !r.eat('{')) return false;
    TuneEntry e;
    if (!r.eat('}')) {
      for (;;) {
        std::string name;
        double v;
        if (!r.str(&name) || !r.eat(':') || !r.num(&v)) return false;
        e.fields[name] = v;
        if (r.eat(',')) continue;
        if (r.eat('}')) break;
        return false;
      }
    }
    parsed[key] = e;
    if (r.eat(',')) continue;
    if (r.eat('}')) break;
    return false;
  }
  for (auto& kv : parsed) entries_[kv.first] = kv.second;
  return true;
}

bool TuneCache::save(const std::string& path) const {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : entries_) {
      f << "  \"" << kv.first << "\": {";
      size_t m = 0;
      for (const auto& fv : kv.second.fields) {
        char buf[64];
        std::snprintf(buf, sizeof(buf), "%.6g", fv.second);
        f << "\"" << fv.first << "\": " << buf << (++m < kv.second.fields.size() ? ", " : "");
      }
      f << "}" << (++n < entries_.size() ? "," : "") << "\n";
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool TuneCache::get(const std::string& key, TuneEntry* out) const {
  auto it = entries_.find(key);
  if (it == entries_.end()) return false;
  *out = it->second;
  return true;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace fockmi
