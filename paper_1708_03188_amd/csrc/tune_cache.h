// Persistent autotuner choices (not ABI): a small text file of
// "key = v0 v1 ..." lines, the key naming the device and the geometry.
#pragma once
#include <string>
#include <vector>

namespace sgm {

// File used: $SGM_TUNE_CACHE if set ("off" disables the file), else
// $XDG_CACHE_HOME/libsgm/tune.txt, else $HOME/.cache/libsgm/tune.txt; "" when
// none applies.
std::string tune_cache_path();
// "<arch>/<compute units>" of the current device (part of every key).
std::string tune_device_tag();
// The last values stored under key (false if none or no file).
bool tune_cache_get(const std::string& key, std::vector<int>& vals);
// Append key = vals (best effort: an unwritable file is ignored).
void tune_cache_put(const std::string& key, const std::vector<int>& vals);

}  // namespace sgm
