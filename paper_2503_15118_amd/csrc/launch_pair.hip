// Launchers of the one-target kernels (compacting k_pair); built once per key
// width W = SS_LW.
#include "kernels.hip"
#include "launch.h"

namespace sparqs {

template <int W, int ITEMS>
static void pair_items(const LaunchCtx& c, int mode, const GroupOp& g, uint32_t ep, uint32_t ep_spec,
                       const FusedRun& run) {
  const uint32_t ntiles = ticket_grid((c.n_ub + kBlock * ITEMS - 1) / (kBlock * ITEMS), c.xo);
  // one child per entry in group mode, two in expand mode
  const uint32_t f = mode == MODE_GROUP ? 1u : 2u;
  KeyPtrs<W> ik, ok;
  for (int w = 0; w < W; ++w) { ik.w[w] = c.in.key[w]; ok.w[w] = c.out.key[w]; }
  if constexpr (W <= 2) {
    if (run.n) {
      if (mode == MODE_GROUP)
        k_pair<W, MODE_GROUP, ITEMS, true><<<ntiles, kBlock, 0, c.stream>>>(
            ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, c.lb, c.meta, ep, c.xo, ep_spec, f, run.ops, run.n, run.gops);
      else
        k_pair<W, MODE_EXPAND, ITEMS, true><<<ntiles, kBlock, 0, c.stream>>>(
            ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, c.lb, c.meta, ep, c.xo, ep_spec, f, run.ops, run.n, run.gops);
      return;
    }
  }
  if (mode == MODE_GROUP)
    k_pair<W, MODE_GROUP, ITEMS, false><<<ntiles, kBlock, 0, c.stream>>>(
        ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, c.lb, c.meta, ep, c.xo, ep_spec, f, nullptr, 0u, nullptr);
  else
    k_pair<W, MODE_EXPAND, ITEMS, false><<<ntiles, kBlock, 0, c.stream>>>(
        ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, c.lb, c.meta, ep, c.xo, ep_spec, f, nullptr, 0u, nullptr);
}

template <int W>
void launch_pair(const LaunchCtx& c, int mode, int items, const GroupOp& g, uint32_t ep, uint32_t ep_spec,
                 const FusedRun& run) {
  if (items >= 4) pair_items<W, 4>(c, mode, g, ep, ep_spec, run);
  else if (items == 2) pair_items<W, 2>(c, mode, g, ep, ep_spec, run);
  else pair_items<W, 1>(c, mode, g, ep, ep_spec, run);
}

template void launch_pair<SS_LW>(const LaunchCtx&, int, int, const GroupOp&, uint32_t, uint32_t, const FusedRun&);

}  // namespace sparqs
