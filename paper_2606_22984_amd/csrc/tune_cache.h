// Persistent store of autotuned launch shapes: a flat JSON object mapping a
// shape key to {"tile": T, "grid": G, "ms": M}, one entry per line, in the file
// named by $FVAN_TUNE_FILE (default $HOME/.cache/fvan_tuning.json; no HOME and
// no FVAN_TUNE_FILE: nothing is persisted).  Writes go to a temporary file
// that replaces the store, so a reader never sees a half-written file.
#pragma once

#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

namespace fvan {

struct TuneEntry {
  int tile = 0, grid = 0;
  double ms = 0.0;
};

inline std::string tune_file_path() {
  if (const char* p = std::getenv("FVAN_TUNE_FILE")) return p;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/fvan_tuning.json";
  return std::string();
}

// Parse lines of the form   "key": {"tile": T, "grid": G, "ms": M},
inline std::map<std::string, TuneEntry> tune_read(const std::string& path) {
  std::map<std::string, TuneEntry> out;
  if (path.empty()) return out;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    char key[512];
    TuneEntry e;
    if (std::sscanf(line, " \"%511[^\"]\": {\"tile\": %d, \"grid\": %d, \"ms\": %lf", key, &e.tile, &e.grid, &e.ms) == 4)
      out[key] = e;
  }
  std::fclose(f);
  return out;
}

inline bool tune_write(const std::string& path, const std::map<std::string, TuneEntry>& entries) {
  if (path.empty()) return false;
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);   // one level
  const std::string tmp = path + ".tmp" + std::to_string((long)std::rand());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : entries) {
    std::fprintf(f, "  \"%s\": {\"tile\": %d, \"grid\": %d, \"ms\": %.4f}%s\n", kv.first.c_str(), kv.second.tile,
                 kv.second.grid, kv.second.ms, ++i < entries.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

inline std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}

}  // namespace fvan
