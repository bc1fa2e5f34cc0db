// The autotuner's cache file: a JSON object
//   {"version": 1, "entries": {"<shape key>": {"<parameter>": <number>, ...}, ...}}
// read and rewritten whole (host code only).
#pragma once

#include <map>
#include <string>

namespace tufrg {

using TuneEntries = std::map<std::string, std::map<std::string, double>>;

// A missing file is an empty cache (true).  A file that exists but is not a
// tuning cache returns false with a message, and must not be overwritten.
bool tune_cache_read(const std::string &path, TuneEntries &out, std::string &err);

// Writes every entry to a temporary file beside path, then renames it over path.
bool tune_cache_write(const std::string &path, const TuneEntries &entries, std::string &err);

}  // namespace tufrg
