// Project autotuner: measured choice of launch variants, cached as JSON.
//
// Keys name the architecture, the precision form and the problem shape; values
// hold the chosen integers and the measured time. The cache file is a flat
// JSON object written by this code only:
//   {"gfx950/fp32/n24/nk64/nb16/nx16": {"variant": 0, "xcd_map": 1, "ms": 89.2}, ...}
#pragma once

#include <map>
#include <string>

namespace fockmi {

struct TuneEntry {
  std::map<std::string, double> fields;  // integer choices are stored as doubles
};

class TuneCache {
 public:
  bool load(const std::string& path);   // false if the file is absent or unreadable
  bool save(const std::string& path) const;
  bool get(const std::string& key, TuneEntry* out) const;
  void put(const std::string& key, const TuneEntry& e) { entries_[key] = e; }
  size_t size() const { return entries_.size(); }

 private:
  std::map<std::string, TuneEntry> entries_;
};

std::string arch_name();  // e.g. "gfx950" for the current device

}  // namespace fockmi
