// Launchers of the LSD radix sort (digit histograms, their scan, scatter
// passes) for every key width.
#include "kernels.hip"
#include "launch.h"

namespace sparqs {

template <int W>
void launch_sort_hist(const LaunchCtx& c, uint32_t nb, const SortPlan& plan, unsigned long long* hist,
                      uint64_t* digit_start) {
  KeyPtrs<W> k;
  for (int w = 0; w < W; ++w) k.w[w] = c.in.key[w];
  k_fill_u64<<<1, kBlock, 0, c.stream>>>(reinterpret_cast<uint64_t*>(hist), (uint64_t)plan.npass * kRadix, 0ull);
  k_sort_hist<W><<<nb, kBlock, plan.npass * kRadix * 4, c.stream>>>(k, c.ns, c.meta, plan, hist);
  k_sort_scan<<<plan.npass, kBlock, 0, c.stream>>>(hist, digit_start);
}

template <int W>
void launch_sort_pass(const LaunchCtx& c, int items, uint32_t ntiles, const PassDesc& pd,
                      const uint64_t* digit_start, uint32_t ep) {
  KeyPtrs<W> ik, ok;
  for (int w = 0; w < W; ++w) { ik.w[w] = c.in.key[w]; ok.w[w] = c.out.key[w]; }
  // with per-XCD tickets the passes take them in chunks of consecutive tiles:
  // a digit's run that one tile ends and the next continues then meets in
  // one XCD's L2 (the scatter writes many such partial lines)
  const uint32_t xo = c.xo ? 2u : 0u;
  ntiles = ticket_grid(ntiles, xo);
  if (items == 16)
    k_sort_pass<W, 16><<<ntiles, kBlock, 0, c.stream>>>(ik, c.in.amp, ok, c.out.amp, c.ns, pd, digit_start, c.lb,
                                                         c.meta, ep, xo);
  else
    k_sort_pass<W, 8><<<ntiles, kBlock, 0, c.stream>>>(ik, c.in.amp, ok, c.out.amp, c.ns, pd, digit_start, c.lb,
                                                        c.meta, ep, xo);
}

template <int W>
static uint32_t hist_resident_w() {
  int dev = 0, per_cu = 0, ncu = 0;
  const size_t lds = (size_t)((64u * W + kMaxGroupBits + kRadixBits - 1) / kRadixBits) * kRadix * 4;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sort_hist<W>, kBlock, lds) != hipSuccess ||
      per_cu <= 0 || ncu <= 0)
    return 0;
  return (uint32_t)per_cu * (uint32_t)ncu;
}

uint32_t sort_hist_resident(uint32_t W) {
  return W == 1 ? hist_resident_w<1>() : W == 2 ? hist_resident_w<2>() : hist_resident_w<4>();
}

template void launch_sort_hist<1>(const LaunchCtx&, uint32_t, const SortPlan&, unsigned long long*, uint64_t*);
template void launch_sort_hist<2>(const LaunchCtx&, uint32_t, const SortPlan&, unsigned long long*, uint64_t*);
template void launch_sort_hist<4>(const LaunchCtx&, uint32_t, const SortPlan&, unsigned long long*, uint64_t*);
template void launch_sort_pass<1>(const LaunchCtx&, int, uint32_t, const PassDesc&, const uint64_t*, uint32_t);
template void launch_sort_pass<2>(const LaunchCtx&, int, uint32_t, const PassDesc&, const uint64_t*, uint32_t);
template void launch_sort_pass<4>(const LaunchCtx&, int, uint32_t, const PassDesc&, const uint64_t*, uint32_t);

}  // namespace sparqs
