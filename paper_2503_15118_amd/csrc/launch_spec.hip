// Launchers of the speculative fixed-placement one-target kernel
// (k_pair_spec); built once per key width W = SS_LW.
#include "kernels.hip"
#include "launch.h"

namespace sparqs {

template <int W, int ITEMS, int NB>
static void spec_wn(const LaunchCtx& c, int mode, const GroupOp& g, uint32_t ep_spec, const FusedRun& run) {
  const uint32_t ntiles = (uint32_t)std::max<uint64_t>(1, (c.n_ub + kBlock * ITEMS - 1) / (kBlock * ITEMS));
  const uint32_t f = mode == MODE_GROUP ? 1u : 2u;
  KeyPtrs<W> ik, ok;
  for (int w = 0; w < W; ++w) { ik.w[w] = c.in.key[w]; ok.w[w] = c.out.key[w]; }
  if constexpr (W <= 2) {
    if (run.n) {
      if (mode == MODE_GROUP)
        k_pair_spec<W, MODE_GROUP, ITEMS, true, NB><<<ntiles, kBlock, 0, c.stream>>>(
            ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, f, c.meta, ep_spec, run.ops, run.n, run.gops);
      else
        k_pair_spec<W, MODE_EXPAND, ITEMS, true, 0><<<ntiles, kBlock, 0, c.stream>>>(
            ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, f, c.meta, ep_spec, run.ops, run.n, run.gops);
      return;
    }
  }
  if (mode == MODE_GROUP)
    k_pair_spec<W, MODE_GROUP, ITEMS, false, NB><<<ntiles, kBlock, 0, c.stream>>>(
        ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, f, c.meta, ep_spec, nullptr, 0u, nullptr);
  else
    k_pair_spec<W, MODE_EXPAND, ITEMS, false, 0><<<ntiles, kBlock, 0, c.stream>>>(
        ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, f, c.meta, ep_spec, nullptr, 0u, nullptr);
}

template <int W, int ITEMS>
static void spec_wi(const LaunchCtx& c, int mode, int nb, const GroupOp& g, uint32_t ep_spec, const FusedRun& run) {
  switch (nb) {
    case 0: spec_wn<W, ITEMS, 0>(c, mode, g, ep_spec, run); break;
    case 2: spec_wn<W, ITEMS, 2>(c, mode, g, ep_spec, run); break;
    default: spec_wn<W, ITEMS, 1>(c, mode, g, ep_spec, run); break;
  }
}

template <int W>
void launch_spec(const LaunchCtx& c, int mode, int items, int nb, const GroupOp& g, uint32_t ep_spec,
                 const FusedRun& run) {
  switch (items) {
    case 1: spec_wi<W, 1>(c, mode, nb, g, ep_spec, run); break;
    case 4: spec_wi<W, 4>(c, mode, nb, g, ep_spec, run); break;
    case 8:
      // 8 entries per thread only where a run is fused and partners sit in
      // neighbouring lanes (one pass over the children): the interpreter's
      // dispatch is then shared by twice the entries
      if constexpr (W <= 2) {
        if (mode == MODE_GROUP && nb == 2 && run.n) {
          constexpr uint32_t T = kBlock * 8;
          const uint32_t ntiles = (uint32_t)std::max<uint64_t>(1, (c.n_ub + T - 1) / T);
          KeyPtrs<W> ik, ok;
          for (int w = 0; w < W; ++w) { ik.w[w] = c.in.key[w]; ok.w[w] = c.out.key[w]; }
          k_pair_spec<W, MODE_GROUP, 8, true, 2><<<ntiles, kBlock, 0, c.stream>>>(
              ik, c.in.amp, ok, c.out.amp, c.ns, c.cap, g, 1u, c.meta, ep_spec, run.ops, run.n, run.gops);
          break;
        }
      }
      spec_wi<W, 4>(c, mode, nb, g, ep_spec, run);
      break;
    default: spec_wi<W, 2>(c, mode, nb, g, ep_spec, run); break;
  }
}

template void launch_spec<SS_LW>(const LaunchCtx&, int, int, int, const GroupOp&, uint32_t, const FusedRun&);

}  // namespace sparqs
