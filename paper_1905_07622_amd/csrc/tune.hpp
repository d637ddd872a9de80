// Autotuner of the gather launch shape: the tile cache (tune_cache.cpp) and
// the shape helpers the search uses (solver.hip, engine.hip).
#pragma once

#include <string>
#include <vector>

#include "common.hpp"

struct fem_heat;

namespace femheat {

// Cache key of a launch shape (see tune_cache.cpp).
std::string tune_key(int device, bool mixed, int kind, bool batched, int px, int py, int pz);
// Tile recorded for `key` in the cache file `path` (false: none).
bool tune_lookup(const char* path, const std::string& key, int tile[3]);
// Records (or replaces) the tile of `key`; false if the file cannot be written.
bool tune_store(const char* path, const std::string& key, const int tile[3], double best_us, double rule_us,
                int candidates);

// Launch shape of a handle's grid with an explicit tile (tz may be 0: the
// library's rule for the handle), and whether its staging scheme holds it.
GatherShape shape_with_tile(const fem_heat* h, int tx, int ty, int tz);
bool shape_stages(const GatherShape& s);
// Candidate shapes of the search for a handle (its own rule first).
std::vector<GatherShape> tune_candidates(const fem_heat* h, int cus);
// Installs a launch shape on a handle, growing its partial-sum buffers when
// the shape has more blocks than they hold.
int set_shape(fem_heat* h, const GatherShape& s);

}  // namespace femheat
