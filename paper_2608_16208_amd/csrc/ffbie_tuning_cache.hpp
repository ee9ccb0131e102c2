// On-disk cache of the batch autotuner's choices (host code).
//
// A JSON file of flat entries, one per (device, M, precision):
//   {"format": "ffbie-tuning-cache", "version": 1, "entries": [
//     {"device": "gfx950 x256", "M": 64, "precision": "f64", "fft_radix": 2,
//      "pairs_per_item": 16, "waves_per_block": 4, "persistent": 0, "main_ms": 1.25},
//     ...]}
// Reading accepts exactly what writing produces (flat objects of string and
// number values inside the "entries" array); anything else leaves the cache
// empty, so a damaged file costs a re-tune, never a wrong launch shape (the
// entries are validated against the launch limits before use).  Writes go to
// a temporary file that is then renamed over the cache.
#pragma once
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ffbie.h"

namespace ffbie {

struct TuneEntry {
  std::string device;
  int M = 0;
  std::string precision;     // "f64" or "f32"
  ffbie_tuning t{};
  double main_ms = 0.0;
};

namespace tune_cache_detail {

inline void skip_ws(const std::string& s, size_t& i) {
  while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
}

inline bool parse_string(const std::string& s, size_t& i, std::string* out) {
  skip_ws(s, i);
  if (i >= s.size() || s[i] != '"') return false;
  ++i;
  out->clear();
  while (i < s.size() && s[i] != '"') {
    if (s[i] == '\\') return false;          // the writer never escapes
    out->push_back(s[i++]);
  }
  if (i >= s.size()) return false;
  ++i;
  return true;
}

inline bool parse_number(const std::string& s, size_t& i, double* out) {
  skip_ws(s, i);
  const char* b = s.c_str() + i;
  char* e = nullptr;
  *out = std::strtod(b, &e);
  if (e == b) return false;
  i += (size_t)(e - b);
  return true;
}

// One flat object {"key": value, ...} at s[i] == '{'.
inline bool parse_entry(const std::string& s, size_t& i, TuneEntry* te) {
  skip_ws(s, i);
  if (i >= s.size() || s[i] != '{') return false;
  ++i;
  int seen = 0;
  while (true) {
    skip_ws(s, i);
    if (i < s.size() && s[i] == '}') { ++i; break; }
    std::string key;
    if (!parse_string(s, i, &key)) return false;
    skip_ws(s, i);
    if (i >= s.size() || s[i] != ':') return false;
    ++i;
    skip_ws(s, i);
    if (key == "device" || key == "precision") {
      std::string v;
      if (!parse_string(s, i, &v)) return false;
      (key == "device" ? te->device : te->precision) = v;
    } else {
      double v;
      if (!parse_number(s, i, &v)) return false;
      if (key == "M") te->M = (int)v;
      else if (key == "fft_radix") te->t.fft_radix = (int)v;
      else if (key == "pairs_per_item") te->t.pairs_per_item = (int)v;
      else if (key == "waves_per_block") te->t.waves_per_block = (int)v;
      else if (key == "persistent") te->t.persistent = (int)v;
      else if (key == "main_ms") te->main_ms = v;
      else return false;
    }
    ++seen;
    skip_ws(s, i);
    if (i < s.size() && s[i] == ',') ++i;
  }
  return seen == 8;
}

}  // namespace tune_cache_detail

// Entries of the cache file at `path` (empty if it is missing or unreadable).
inline std::vector<TuneEntry> tune_cache_read(const std::string& path) {
  std::vector<TuneEntry> out;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return out;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  std::fclose(f);
  if (s.find("\"ffbie-tuning-cache\"") == std::string::npos) return out;
  size_t i = s.find("\"entries\"");
  if (i == std::string::npos) return out;
  i = s.find('[', i);
  if (i == std::string::npos) return out;
  ++i;
  while (true) {
    tune_cache_detail::skip_ws(s, i);
    if (i >= s.size()) return {};
    if (s[i] == ']') break;
    TuneEntry te;
    if (!tune_cache_detail::parse_entry(s, i, &te)) return {};
    out.push_back(te);
    tune_cache_detail::skip_ws(s, i);
    if (i < s.size() && s[i] == ',') ++i;
  }
  return out;
}

inline const TuneEntry* tune_cache_find(const std::vector<TuneEntry>& v, const std::string& device,
                                        int M, const std::string& precision) {
  for (const TuneEntry& e : v)
    if (e.device == device && e.M == M && e.precision == precision) return &e;
  return nullptr;
}

// Writes `v` to `path` (through path + ".tmp" and a rename).  Returns false on
// an I/O error.
inline bool tune_cache_write(const std::string& path, const std::vector<TuneEntry>& v) {
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{\"format\": \"ffbie-tuning-cache\", \"version\": 1, \"entries\": [\n");
  for (size_t k = 0; k < v.size(); ++k) {
    const TuneEntry& e = v[k];
    std::fprintf(f,
                 "  {\"device\": \"%s\", \"M\": %d, \"precision\": \"%s\", \"fft_radix\": %d, "
                 "\"pairs_per_item\": %d, \"waves_per_block\": %d, \"persistent\": %d, "
                 "\"main_ms\": %.6g}%s\n",
                 e.device.c_str(), e.M, e.precision.c_str(), e.t.fft_radix, e.t.pairs_per_item,
                 e.t.waves_per_block, e.t.persistent, e.main_ms, k + 1 < v.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok) return false;
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace ffbie
