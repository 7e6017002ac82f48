// Packed symmetric Kerr contraction on matrix cores (placeholder until the
// MFMA kernel lands; the plan never selects this path yet).
#include "common.h"

namespace mmnlse {

hipError_t launch_kerr_mfma(const Plan &, double, const KerrLaunch &) { return hipErrorNotSupported; }

hipError_t launch_pack_bf16(const Plan &) { return hipErrorNotSupported; }

hipError_t setup_mfma(Plan &, const float *) { return hipErrorNotSupported; }

}  // namespace mmnlse
