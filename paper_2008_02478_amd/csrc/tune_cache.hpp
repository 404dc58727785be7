// Schedule cache of the launch-shape tuner: a small JSON file that maps a
// key (device, mesh or layer-group geometry, batch size) to the chosen
// launch shape and the times that were measured for it.
//
//   {"format": "demag-schedule-cache/1",
//    "entries": {"<key>": {"yg": 2, "kw": 4, "radix": 8, "zsep": 0, "x_us": 190.0, "mid_us": 230.5}, ...}}
//
// Host code only; no HIP calls.
#pragma once
#include <map>
#include <string>

namespace demag {

struct TuneEntry {
  int yg = 0;        // y rows per workgroup of the x passes (0: not tuned)
  int kw = 0;        // kx lines per workgroup of the middle pass
  int radix = 0;     // points per lane of its y line FFT
  int zsep = -1;     // 1: separate z passes, 0: fused x+z passes (-1: not recorded)
  double x_us = 0;   // measured time of the x passes (forward + inverse)
  double mid_us = 0; // measured time of the middle pass(es)
};

using TuneMap = std::map<std::string, TuneEntry>;

// Reads the cache at `path` into `out`.  A missing file is an empty cache.
// Returns false (with a message in err) for an unreadable or malformed file.
bool tune_cache_read(const std::string& path, TuneMap& out, std::string& err);

// Writes `m` to `path` through a temporary file and a rename.
bool tune_cache_write(const std::string& path, const TuneMap& m, std::string& err);

// Parses cache text (exposed for the reader; false on malformed input).
bool tune_cache_parse(const std::string& text, TuneMap& out, std::string& err);

}  // namespace demag
