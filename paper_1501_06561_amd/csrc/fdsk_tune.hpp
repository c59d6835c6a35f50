// Launch-shape tuner: for a product kernel with several valid launch shapes
// (the Gram's split-K count, the rebuild's rows per workgroup), the shape is
// chosen per bucket of sizes by timing every candidate on the device once and
// keeping the fastest.  Choices are kept per process in a table keyed by a
// string that names the device, the product, the precision and the size
// bucket, and persisted to a text cache file (one "key<TAB>value" line per
// choice), so that later processes on the same kind of device reuse them
// without timing.
//
// Every candidate computes the same product; the choice changes the order in
// which partial sums are added (split-K) and nothing else, so results differ
// between choices by rounding only.  With tuning off, the fixed default of
// each launch is used.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

namespace fdsk {

enum TuneMode { TUNE_OFF = 0, TUNE_ON = 1, TUNE_REFRESH = 2 };

// Current mode: FDSK_TUNE in the environment at first use ("0"/"off",
// "1"/"on", "refresh"; default on), or what fdsk_tune_set_mode set.
int tune_mode();

// "<arch>/<compute units>" of the current device, the prefix of every key.
std::string tune_device_tag();

// Smallest power of two >= x (x >= 1), for size buckets.
int tune_bucket(int x);

// The tuned value of key, or dflt when tuning is off.  On a miss (or in
// refresh mode) every candidate is run through launch(c) on stream s -- one
// warm-up, then `reps` timed launches between two events -- and the fastest
// is recorded (the default wins unless another is at least 3% faster).  A
// candidate whose launch fails is skipped; when all fail, dflt is returned
// and nothing is recorded.  The stream is synchronised; the launches write
// whatever the product writes, so callers tune on workspaces whose contents
// do not matter yet.
int tune_pick(const std::string& key, const std::vector<int>& candidates, int dflt, hipStream_t s,
              const std::function<hipError_t(int)>& launch, int reps = 5);

}  // namespace fdsk
