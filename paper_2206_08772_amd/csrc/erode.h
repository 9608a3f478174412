// Erosion launcher of libotm (not exported).
#pragma once

#include "launch.h"

namespace otm {

// Removes the MPs flagged in st.failed from every per-MP array (stable
// order; component stride becomes the survivor count) and sets st.n_mp.
// Synchronises the stream once, to read the survivor count.
otm_status launch_erode(otm_state& st, const Workspace& w, hipStream_t s);

}  // namespace otm
