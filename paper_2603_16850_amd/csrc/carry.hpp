// The carry pass that completes a diagonal scan after the per-group pass, shared by the GRU
// quasi-DEER forward iteration and the adjoint iteration.
//
// The per-group pass leaves, for every step t and unit d, the map composed from the first
// scanned step of t's group to t:  Delta_t = la_t Delta_in + lc_t  ((la_t, lc_t) stored per
// step), and the group's whole map (agg[group][d]).  With the groups of a sequence numbered
// by scan order (group slots group_start[b] .. group_start[b+1]-1):
//   carry[first] = 0,  carry[g+1] = agg_a[g] carry[g] + agg_c[g]   (eq. bin_op_affine)
// and the next iteration's per-group pass applies  out_t = in_t + la_t carry[group(t)] + lc_t.
#pragma once
#include "pn_host.hpp"

namespace pn {

// Scan of the group maps, one wave per (sequence, 4 units).  Sequences whose status is not
// active are skipped; nothing runs when ctrl->all_done is set.  With grmax ([ngroups][nw]
// residual maxima of the groups' waves, float bits) the sequence's converged prefix of groups
// is frozen (SeqState::frozen) and the scan restarts after it.
void launch_carry_scan(const float2* agg, float* carry, const IterState& st, int B, int D,
                       hipStream_t stream, const uint32_t* grmax = nullptr, int nw = 0);

}  // namespace pn
