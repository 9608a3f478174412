// Erosion launcher of libotm (not exported).
#pragma once

#include "launch.h"

namespace otm {

// Removes the MPs flagged in st.failed from every per-MP array (stable
// order; component stride becomes the survivor count) and sets st.n_mp.
// With p.insert_dist > 0, first appends a node at each removed MP that has
// no node within insert_dist and no removed MP of smaller index within it
// (node arrays re-strided to the new st.n_nodes; *inserted receives the
// count).  Synchronises the stream to read the counts.
otm_status launch_erode(otm_state& st, const otm_params& p, const Workspace& w, hipStream_t s,
                        int64_t* inserted);

// Removes the nodes that no pair uses from every node array (stable order),
// renumbers the support lists and sets st.n_nodes; *deleted receives the
// count.  Synchronises the stream.
otm_status launch_delete_orphans(otm_state& st, const otm_params& p, const Workspace& w,
                                 hipStream_t s, int64_t* deleted);

}  // namespace otm
