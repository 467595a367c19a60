// Launchers of the kernels for ops on 2..10 target qubits (k_group,
// k_expand_slots); built once per key width W = SS_LW.
#include "kernels.hip"
#include "launch.h"

namespace sparqs {

template <int W, int K, int ITEMS>
static void multi_wki(const LaunchCtx& c, int mode, bool slots, const GroupOp& g, uint32_t ep) {
  KeyPtrs<W> ik, ok;
  for (int w = 0; w < W; ++w) { ik.w[w] = c.in.key[w]; ok.w[w] = c.out.key[w]; }
  if (K > kMaxGroupBits || (mode == MODE_EXPAND && slots)) {
    // one thread per child: 2^K slots per entry, 4 per thread (more than
    // kMaxGroupBits targets come here only as pure expansions that fit)
    constexpr uint32_t kSlotTile = kBlock * 4;
    const uint64_t nslots = c.n_ub << K;
    const uint32_t nt = ticket_grid((nslots + kSlotTile - 1) / kSlotTile, c.xo);
    k_expand_slots<W, K, 4><<<nt, kBlock, 0, c.stream>>>(ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, c.lb, c.meta,
                                                         ep, c.xo);
    return;
  }
  if constexpr (K <= kMaxGroupBits) {
    const uint32_t ntiles = ticket_grid((c.n_ub + kBlock * ITEMS - 1) / (kBlock * ITEMS), c.xo);
    if (mode == MODE_GROUP)
      k_group<W, K, MODE_GROUP, ITEMS><<<ntiles, kBlock, 0, c.stream>>>(ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g,
                                                                        c.lb, c.meta, ep, c.xo);
    else
      k_group<W, K, MODE_EXPAND, ITEMS><<<ntiles, kBlock, 0, c.stream>>>(ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g,
                                                                         c.lb, c.meta, ep, c.xo);
  }
}

// Items per thread: several for two targets (bigger tiles, fewer tile-id
// atomics), one for 8..32-member groups (register budget).
template <int W, int K>
static void multi_wk(const LaunchCtx& c, int mode, int items, bool slots, const GroupOp& g, uint32_t ep) {
  if (K <= 2 && items >= 4) multi_wki<W, K, (K <= 2 ? 4 : 1)>(c, mode, slots, g, ep);
  else if (K <= 2 && items == 2) multi_wki<W, K, (K <= 2 ? 2 : 1)>(c, mode, slots, g, ep);
  else multi_wki<W, K, 1>(c, mode, slots, g, ep);
}

template <int W>
void launch_multi(const LaunchCtx& c, int mode, int items, bool slots, const GroupOp& g, uint32_t ep) {
  switch (g.k) {
    case 2: multi_wk<W, 2>(c, mode, items, slots, g, ep); break;
    case 3: multi_wk<W, 3>(c, mode, items, slots, g, ep); break;
    case 4: multi_wk<W, 4>(c, mode, items, slots, g, ep); break;
    case 5: multi_wk<W, 5>(c, mode, items, slots, g, ep); break;
    case 6: multi_wk<W, 6>(c, mode, items, slots, g, ep); break;
    case 7: multi_wk<W, 7>(c, mode, items, slots, g, ep); break;
    case 8: multi_wk<W, 8>(c, mode, items, slots, g, ep); break;
    case 9: multi_wk<W, 9>(c, mode, items, slots, g, ep); break;
    default: multi_wk<W, 10>(c, mode, items, slots, g, ep); break;
  }
}

template void launch_multi<SS_LW>(const LaunchCtx&, int, int, bool, const GroupOp&, uint32_t);

}  // namespace sparqs
