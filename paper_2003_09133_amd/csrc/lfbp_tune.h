// Tuned kernel choices for the H -> H' re-arrangement.
#pragma once

#include "lfbp.h"

namespace lfbp {

// The configuration for one problem: an entry of the tuning table when one
// matches (dtype, W = ny*nz, nx), else the built-in defaults.  Every field is
// set (grid may be 0 = one workgroup per work unit).
lfbp_gather_config tuned_config(const lfbp_shape& s, int esize);

}  // namespace lfbp
