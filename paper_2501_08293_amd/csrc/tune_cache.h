// Persistent cache of autotuner decisions (internal header; see tune_cache.cpp).
#pragma once

#include <string>
#include <vector>

namespace opf {

// The values stored for `key`, if any (false when absent or unreadable).
bool tune_cache_get(const std::string& key, std::vector<int>& vals);
// Stores the values for `key` (a failure to write only disables the cache).
void tune_cache_put(const std::string& key, const std::vector<int>& vals);

}  // namespace opf
