// In-process autotuner of launch variants (tune.hip).
#pragma once
#include <functional>
#include <string>

#include <hip/hip_runtime.h>

namespace awg {
// Cached variant for key, or -1 when not measured yet (0 when tuning is off).
int tune_lookup(const std::string& key);
// Index of the fastest of nvar variants for key; run(v) launches variant v on
// stream s (each variant must write the same result).  Measures on first use.
int tune_pick(const std::string& key, int nvar, const std::function<void(int)>& run, hipStream_t s);
void tune_enable(bool on);
std::string tune_json();
}  // namespace awg
