// Subtree kernel: placeholder until the single-launch latency path lands.
#include "cyrus_device.h"
#include "cyrus_host.h"

namespace cyrus {

bool subtree_supported(const DevTree&, int) { return false; }

hipError_t launch_subtree(const DevTree&, int, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace cyrus
