// Launchers of the fused non-branching run (k_perm_fast for keys of 1 or 2
// words, k_perm for 4); built once per key width W = SS_LW.
#include "kernels.hip"
#include "launch.h"

namespace sparqs {

template <int W, int E>
static void perm_fast(const LaunchCtx& c, bool amp, const FastOp* f, uint32_t nfast, const PermOp* gops,
                      uint32_t write_words, uint32_t ep) {
  KeyPtrs<W> k;
  for (int w = 0; w < W; ++w) k.w[w] = c.in.key[w];
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, (c.n_ub + kBlock * E - 1) / (kBlock * E));
  if (amp)
    k_perm_fast<W, E, true><<<grid, kBlock, 0, c.stream>>>(k, c.in.amp, c.ns, f, nfast, gops, write_words, c.meta, ep);
  else
    k_perm_fast<W, E, false><<<grid, kBlock, 0, c.stream>>>(k, c.in.amp, c.ns, f, nfast, gops, write_words, c.meta,
                                                            ep);
}

template <int W>
void launch_perm(const LaunchCtx& c, int e, bool amp, const FastOp* f, uint32_t nfast, const PermOp* gops,
                 uint32_t write_words, uint32_t ep) {
  if constexpr (W <= 2) {
    if (e == 16) perm_fast<W, 16>(c, amp, f, nfast, gops, write_words, ep);
    else if (e == 8) perm_fast<W, 8>(c, amp, f, nfast, gops, write_words, ep);
    else perm_fast<W, 4>(c, amp, f, nfast, gops, write_words, ep);
  } else {
    KeyPtrs<W> k;
    for (int w = 0; w < W; ++w) k.w[w] = c.in.key[w];
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((c.n_ub + kBlock - 1) / kBlock, 8192));
    if (amp)
      k_perm<W, true><<<grid, kBlock, 0, c.stream>>>(k, c.in.amp, c.ns, gops, nfast, write_words, c.meta, ep);
    else
      k_perm<W, false><<<grid, kBlock, 0, c.stream>>>(k, c.in.amp, c.ns, gops, nfast, write_words, c.meta, ep);
  }
}

template void launch_perm<SS_LW>(const LaunchCtx&, int, bool, const FastOp*, uint32_t, const PermOp*, uint32_t,
                                 uint32_t);

}  // namespace sparqs
