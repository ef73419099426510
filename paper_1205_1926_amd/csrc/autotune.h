// Autotuner cache of the F-apply launch parameters: a text file of JSON
// lines keyed by (GPU architecture, factor precision, histogram of the
// subdomain sizes).  Host code only.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tfeti {

struct TuneChoice {
  int tile = 32;      // rows per factor tile: 16, 32 or 64
  int natural = 0;    // subdomain schedule: 0 longest first, 1 natural order
  int threads = 256;  // threads per workgroup of the subdomain solves: 256, 512 or 1024
  double ms = 0.0;    // median F-apply time measured for this choice
};

// Key of a problem: "<arch>|<fp64|fp32>|n=<subdomains>|h=<hash of the sorted
// (DOF count, multiplicity) list>".
std::string tune_key(const std::string& arch, int precision, const std::vector<int32_t>& ndofs);

// Look the key up in the cache file; false if the file or the key is absent
// or the entry is malformed.
bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice* out);

// Insert or replace the key's entry (the file is rewritten whole); false if
// it cannot be written.
bool tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c);

}  // namespace tfeti
