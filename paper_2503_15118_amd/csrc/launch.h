// Host-side launchers of the large kernel families.  Each family is compiled
// in its own translation unit (and, for the emitting kernels, once per key
// width), so the device code of the library builds in parallel; the planner
// in sparqs.hip calls these with plain arguments.
#pragma once

#include "sparqs_internal.h"

#include <algorithm>

namespace sparqs {

// Key-word arrays and amplitude array of one entry buffer (SoA).
struct Buf {
  uint64_t* key[kMaxW];
  double2* amp;
};

// A run of non-branching ops fused into a one-target launch (n == 0: none).
struct FusedRun {
  const FastOp* ops;
  uint32_t n;
  const PermOp* gops;
};

// What every launcher needs of the state: its stream, the buffer read (in)
// and written (out), the count slot read, the capacity, the host's bound on
// the entry count (grid size), look-back words, meta block and tile order.
struct LaunchCtx {
  hipStream_t stream;
  Buf in, out;
  uint32_t ns;
  uint64_t cap, n_ub;
  uint64_t* lb;
  DevMeta* meta;
  uint32_t xo;
};

// Grid of a launch whose workgroups take tile tickets: with chunked tickets
// (xo == 2) every workgroup takes one, so the grid is a whole number of
// 8 x kTileChunk workgroups.
inline uint32_t ticket_grid(uint64_t ntiles, uint32_t xo) {
  uint64_t g = std::max<uint64_t>(1, ntiles);
  if (xo == 2) {
    const uint64_t q = (uint64_t)kXcds * kTileChunk;
    g = (g + q - 1) / q * q;
  }
  return (uint32_t)g;
}

// One-target op with compaction (k_pair): items entries per thread (1|2|4).
template <int W>
void launch_pair(const LaunchCtx& c, int mode, int items, const GroupOp& g, uint32_t ep, uint32_t ep_spec,
                 const FusedRun& run);

// One-target op at fixed positions, no look-back (k_pair_spec); nb selects how
// group-mode partners are found (0 staged, 1 lane pair with staging fallback,
// 2 lane pair only).
template <int W>
void launch_spec(const LaunchCtx& c, int mode, int items, int nb, const GroupOp& g, uint32_t ep_spec,
                 const FusedRun& run);

// Ops on 2..kMaxExpandBits targets: k_group (butterflies, up to kMaxGroupBits)
// or k_expand_slots (one thread per child; expansions only).
template <int W>
void launch_multi(const LaunchCtx& c, int mode, int items, bool slots, const GroupOp& g, uint32_t ep);

// Fused run of non-branching ops in place on buffer `in`: the 32-bit
// interpreter (W <= 2, e entries per lane) or the generic 64-bit one (W = 4).
template <int W>
void launch_perm(const LaunchCtx& c, int e, bool amp, const FastOp* f, uint32_t nfast, const PermOp* gops,
                 uint32_t write_words, uint32_t ep);

// Radix sort: all-pass digit histograms (nb workgroups adding into one global
// histogram per pass, np x 256 u64 at `hist`), their scan, and one
// scatter pass from `in` to `out` over ntiles tiles of kBlock*items entries.
template <int W>
void launch_sort_hist(const LaunchCtx& c, uint32_t nb, const SortPlan& plan, unsigned long long* hist,
                      uint64_t* digit_start);
// Workgroups of the histogram kernel for W-word keys that the current device
// holds at once (occupancy at the largest histogram area x compute units);
// 0 when the runtime cannot say.
uint32_t sort_hist_resident(uint32_t W);
template <int W>
void launch_sort_pass(const LaunchCtx& c, int items, uint32_t ntiles, const PassDesc& pd,
                      const uint64_t* digit_start, uint32_t ep);

}  // namespace sparqs
