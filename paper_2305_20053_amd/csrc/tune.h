// Persisted autotuning choices (launch shapes picked by timing at first use).
#pragma once
#include <string>

namespace saa_tune {

// The recorded choice for `key` on the current device, or -1.  Keys name the
// kernel, its precision and the problem size; the device (architecture and
// compute-unit count) is prefixed here.
int lookup(const std::string& key);

// Record a choice (kept in memory and appended to the cache file).
void store(const std::string& key, int value);

// The cache file: $SAA_TUNE_CACHE if set ("off": memory only), else
// $HOME/.cache/saa_tune.txt (memory only without HOME).  One "key value" pair
// per line; the last line of a key wins.
std::string path();

}  // namespace saa_tune
