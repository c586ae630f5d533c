// On-disk cache of the autotuner's choices (host code).
//
// The tuner times the result-invariant variants of a plan's dominant kernel
// (operand prefetch distance, wave height, queue placement) on a short run of
// the caller's own shape, and keeps the fastest per key.  The key names the
// device architecture, the plan, the variant and the padded shape.
#pragma once
#include <string>
#include <vector>

namespace hsb {

// The cache file: $HSB_TUNE_CACHE, else $XDG_CACHE_HOME/hsb/tune.txt, else
// $HOME/.cache/hsb/tune.txt, else ./hsb_tune.txt.
std::string tune_cache_path();
// The stored choice of `key`, if any.
bool tune_lookup(const std::string &key, int *choice);
// Store (replace) the choice of `key` with the times measured per candidate.
// Returns false if the file could not be written (the choice is still kept
// for the rest of the process).
bool tune_store(const std::string &key, int choice, const std::vector<double> &ms);

}  // namespace hsb
