// Tuned kernel choices for the H -> H' re-arrangement.
#pragma once

#include "lfbp.h"

namespace lfbp {

// The configuration for one problem: an entry of the tuning table when one
// matches (batched or plain, element size, W = ny*nz, nx), else the built-in
// defaults.  Every field is set except grid, which may be 0 (= one workgroup
// per unit, or every workgroup slot of the device when persistent).
lfbp_gather_config tuned_config(const lfbp_shape& s, int esize, bool batched);

}  // namespace lfbp
