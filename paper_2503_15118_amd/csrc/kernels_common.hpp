// Wave64 / workgroup primitives and decoupled look-back for gfx950.
#pragma once

#include "sparqs_internal.h"

namespace sparqs {

template <int W>
struct KeyPtrs {
  uint64_t* w[W];
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `m` in lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += t;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_and(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v &= __shfl_xor(v, d, 64);
  return v;
}

// Exclusive scan over the 256 threads of a workgroup; `lds` holds 4 values.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T& total) {
  T inc = wave_incl_scan(v);
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) lds[w] = inc;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < kBlock / 64; ++i) {
    T x = lds[i];
    if (i < w) pre += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return pre + inc - v;
}

constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ bool lb_ready(uint64_t v, uint32_t epoch) {
  return ((uint32_t)(v >> kLbEpochShift) == (epoch & kEpochMask)) && (v & kLbFlagMask);
}

// Decoupled look-back for one running total per tile, executed by every lane
// of one wave.  Publishes `agg` for `tile`, returns the sum over all earlier
// tiles (identical on every lane) and publishes the inclusive total.  A wait
// that exceeds kSpinLimit polls raises kErrSpin and gives up (the result is
// then wrong but every wave exits).
__device__ uint64_t lookback_single(uint64_t* lb, uint32_t tile, uint64_t agg, uint32_t epoch,
                                    unsigned int* err) {
  const uint64_t ep = (uint64_t)(epoch & kEpochMask) << kLbEpochShift;
  const uint32_t lane = lane_id();
  if (tile == 0) {
    if (lane == 0) st_agent(&lb[0], ep | kLbInc | agg);
    return 0;
  }
  if (lane == 0) st_agent(&lb[tile], ep | kLbAgg | agg);
  uint64_t excl = 0;
  int64_t top = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (true) {
    const int64_t idx = top - (int64_t)lane;
    const uint64_t v = idx >= 0 ? ld_agent(&lb[idx]) : (ep | kLbInc);
    const bool rd = lb_ready(v, epoch);
    const uint64_t rdy = __ballot(rd);
    const uint64_t inc = __ballot(rd && (v & kLbInc));
    const uint32_t first_nr = (~rdy) ? (uint32_t)__builtin_ctzll(~rdy) : 64u;
    const uint32_t first_inc = inc ? (uint32_t)__builtin_ctzll(inc) : 64u;
    if (first_inc < first_nr) {
      excl += wave_sum<uint64_t>(lane <= first_inc ? (v & kLbValueMask) : 0ull);
      break;
    }
    if (first_nr == 64u) {
      excl += wave_sum<uint64_t>(v & kLbValueMask);
      top -= 64;
      continue;
    }
    if (++spins > kSpinLimit) {
      if (lane == 0) atomicOr(err, kErrSpin);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (lane == 0) st_agent(&lb[tile], ep | kLbInc | (excl + agg));
  return excl;
}

// Exclusive prefix of a tile's count for a whole workgroup: wave 0 runs the
// look-back (64 predecessor words per round trip), the others wait at the
// barrier.  A block-wide 256-word window was measured slower: four barriers
// per round cost more than the round trips it saves.
__device__ uint64_t lookback_block(uint64_t* lb, uint32_t tile, uint64_t agg, uint32_t epoch,
                                   unsigned int* err, uint64_t* s) {
  if ((threadIdx.x >> 6) == 0) {
    const uint64_t excl = lookback_single(lb, tile, agg, epoch, err);
    if (threadIdx.x == 0) s[0] = excl;
  }
  __syncthreads();
  return s[0];
}

// Per-digit look-back: thread `d` of the workgroup walks its own chain,
// reading 8 predecessors per round trip.
__device__ uint64_t lookback_digit(uint64_t* lb, uint32_t tile, uint32_t d, uint64_t cnt,
                                   uint32_t epoch, unsigned int* err) {
  constexpr int B = 8;
  const uint64_t ep = (uint64_t)(epoch & kEpochMask) << kLbEpochShift;
  uint64_t* row = lb + (uint64_t)tile * kRadix;
  if (tile == 0) {
    st_agent(&row[d], ep | kLbInc | cnt);
    return 0;
  }
  st_agent(&row[d], ep | kLbAgg | cnt);
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (true) {
    uint64_t v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int64_t k = j - b;
      v[b] = k >= 0 ? ld_agent(&lb[(uint64_t)k * kRadix + d]) : (ep | kLbInc);
    }
    // accept the longest ready prefix; stop at the first inclusive total
    int used = 0;
    bool found = false;
    uint64_t part = 0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (found || used < b) continue;
      if (!lb_ready(v[b], epoch)) continue;
      part += v[b] & kLbValueMask;
      used = b + 1;
      if (v[b] & kLbInc) found = true;
    }
    excl += part;
    j -= used;
    if (found) break;
    if (used == 0) {
      if (++spins > kSpinLimit) {
        atomicOr(err, kErrSpin);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  st_agent(&row[d], ep | kLbInc | (excl + cnt));
  return excl;
}

__device__ __forceinline__ uint32_t xcc_id() {
  // HW_REG_XCC_ID (id 20), bits [3:0]
  return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 15u;
}

// Dynamic tile id.  With `xcd_order` (one stream; the device sends workgroups
// with equal blockIdx % 8 to one XCD and distinct residues to distinct XCDs,
// checked when the state is created) residue class x has its own counter and
// its k-th workgroup to start takes tile 8k + x: the counters see 8x less
// contention, and a tile waits only on lower tiles, each taken by a running
// workgroup or by one that its XCD will still start.  Otherwise one counter
// hands out tiles in start order.
// xcd_order 1: XCD x (workgroups spread round robin over the 8 XCDs) hands
// out tiles x, x + 8, ... from its own counter.  2: tickets in chunks per
// XCD: XCD x hands out, in order, the tiles whose index / kTileChunk is x
// modulo 8, so kTileChunk consecutive tiles run on one XCD and what they share
// (the output lines where one tile's writes end and the next one's begin, the
// next tile's look-back words) meets in that XCD's L2.  With 2 every workgroup
// of the grid (a multiple of 8 x kTileChunk) takes a ticket and those past the
// tile count leave (tile_out_of_range).
__device__ __forceinline__ uint32_t take_tile(DevMeta* meta, uint32_t epoch, uint32_t* s_tile,
                                              uint32_t xcd_order) {
  if (threadIdx.x == 0) {
    const uint32_t slot = epoch % kRing;
    uint32_t t;
    if (xcd_order == 2) {
      const uint32_t x = blockIdx.x % kXcds;
      const uint32_t k = (uint32_t)atomicAdd(&meta->xcd_ctr[slot][x * kXcdStride], 1ull);
      t = ((k / kTileChunk) * kXcds + x) * kTileChunk + k % kTileChunk;
    } else if (xcd_order) {
      const uint32_t x = blockIdx.x % kXcds;
      t = (uint32_t)atomicAdd(&meta->xcd_ctr[slot][x * kXcdStride], 1ull) * kXcds + x;
    } else {
      t = (uint32_t)atomicAdd(&meta->counters[slot], 1ull);
    }
    *s_tile = t;
  }
  __syncthreads();
  return *s_tile;
}

// Launch prologue of every kernel that owns an epoch: workgroup 0 clears the
// ring slot a launch kRing/2 epochs later will use.  Returns true (the same
// value in every thread of the workgroup) when an earlier launch raised an
// error: the kernel then changes nothing, and the host rolls the state back to
// the input of the failing launch.
__device__ __forceinline__ bool launch_prologue(DevMeta* meta, uint32_t epoch) {
  __shared__ unsigned int s_err;
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) {
      const uint32_t r = (epoch + kRing / 2) % kRing;
      meta->counters[r] = 0;
      meta->spec_irr[r] = 0;
      for (int x = 0; x < kXcds; ++x) meta->xcd_ctr[r][x * kXcdStride] = 0;
      meta->nnz_out[r] = 0;
      for (int w = 0; w < kMaxW; ++w) {
        meta->or_mask[r][w] = 0;
        meta->and_mask[r][w] = ~0ull;
      }
    }
    s_err = *reinterpret_cast<volatile unsigned int*>(&meta->err);
  }
  __syncthreads();
  return s_err != 0u;
}

// launch_prologue that also reads, in the same round trip as the error word,
// the entry count of ring slot `ns`, the view base (batched rounds, when
// `view`) and one more flag word (when `flag` is not null).  Thread 0 issues
// the loads together (relaxed agent-scope loads: unlike volatile ones they
// are not each waited for) and the workgroup takes the values from LDS.
struct PrologueReads {
  uint64_t n, base;
  unsigned int flag;
};
__device__ __forceinline__ bool launch_prologue_reads(DevMeta* meta, uint32_t epoch, uint32_t ns, bool view,
                                                      unsigned int* flag, PrologueReads* out) {
  __shared__ unsigned int s_err2, s_flag;
  __shared__ uint64_t s_n, s_base;
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) {
      const uint32_t r = (epoch + kRing / 2) % kRing;
      meta->counters[r] = 0;
      meta->spec_irr[r] = 0;
      for (int x = 0; x < kXcds; ++x) meta->xcd_ctr[r][x * kXcdStride] = 0;
      meta->nnz_out[r] = 0;
      for (int w = 0; w < kMaxW; ++w) {
        meta->or_mask[r][w] = 0;
        meta->and_mask[r][w] = ~0ull;
      }
    }
    const unsigned int e = __hip_atomic_load(&meta->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t n = __hip_atomic_load(&meta->nring[ns & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = view ? __hip_atomic_load(&meta->base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
    const unsigned int f = flag ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    s_err2 = e;
    s_n = n;
    s_base = b;
    s_flag = f;
  }
  __syncthreads();
  out->n = s_n;
  out->base = s_base;
  out->flag = s_flag;
  return s_err2 != 0u;
}

__device__ __forceinline__ void raise_error(DevMeta* meta, uint32_t bits, uint32_t epoch) {
  atomicOr(&meta->err, bits);
  atomicCAS(&meta->err_epoch, 0u, epoch);
}

// Start of an emitting launch that reads its entry count from ring slot `ns`
// and writes the output count to the other slot.  Grids are sized from an
// upper bound of the count: a workgroup past the count's tiles leaves before
// taking a tile ticket, so tickets go to exactly ceil(n / tile) workgroups.
// Returns false when the workgroup has nothing to do (an earlier error, an
// empty input: workgroup 0 then records an empty output, or excess).  A grid
// smaller than the count is flagged rather than leaving entries behind.
// `flag` (optional): a word read in the prologue's round trip, into *flag_out.
__device__ __forceinline__ bool emit_begin(DevMeta* meta, uint32_t ns, uint32_t epoch, uint64_t tile_entries,
                                           uint64_t* n_out, uint32_t xcd_order, unsigned int* flag = nullptr,
                                           unsigned int* flag_out = nullptr) {
  PrologueReads pr;
  if (launch_prologue_reads(meta, epoch, ns, false, flag, &pr)) return false;
  const uint64_t n = pr.n;
  *n_out = n;
  if (flag_out) *flag_out = pr.flag;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (n == 0) {
      meta->nring[(ns & 1) ^ 1] = 0;
      meta->nnz_out[epoch % kRing] = 0;
    }
    if ((uint64_t)gridDim.x * tile_entries < n) raise_error(meta, kErrGrid, epoch);
  }
  return xcd_order == 2 || (uint64_t)blockIdx.x * tile_entries < n;
}

// emit_begin on the view [base, n) of batched rounds: the count returned is
// n - base (positions are relative to base); an empty view records the
// unchanged total as the output count.
__device__ __forceinline__ bool emit_begin_view(DevMeta* meta, uint32_t ns, uint32_t epoch, uint64_t tile_entries,
                                                uint64_t* n_out, uint64_t* base_out, uint32_t xcd_order) {
  PrologueReads pr;
  if (launch_prologue_reads(meta, epoch, ns, true, nullptr, &pr)) return false;
  const uint64_t base = pr.base;
  const uint64_t n = pr.n - base;
  *n_out = n;
  *base_out = base;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (n == 0) {
      meta->nring[(ns & 1) ^ 1] = base;
      meta->nnz_out[epoch % kRing] = base;
    }
    if ((uint64_t)gridDim.x * tile_entries < n) raise_error(meta, kErrGrid, epoch);
  }
  return xcd_order == 2 || (uint64_t)blockIdx.x * tile_entries < n;
}

template <int W>
__device__ __forceinline__ void offset_keys(KeyPtrs<W>& k, uint64_t off) {
#pragma unroll
  for (int w = 0; w < W; ++w) k.w[w] += off;
}

// A tile id at or past the tile count cannot be handed out when only
// workgroups inside the count take tickets; such a workgroup touches nothing.
__device__ __forceinline__ bool tile_out_of_range(uint32_t tile, uint64_t ntiles, unsigned int* err,
                                                  uint32_t xcd_order) {
  if (tile < ntiles) return false;
  // chunked tickets hand out every tile of the grid: those past the count leave
  if (xcd_order != 2 && threadIdx.x == 0) atomicOr(err, kErrGrid);
  return true;
}

template <int W>
__device__ __forceinline__ void publish_masks(DevMeta* meta, uint32_t epoch, const uint64_t (&orv)[W],
                                              const uint64_t (&andv)[W], uint64_t* s_red) {
  // s_red: 2*W*4 values of LDS
  const uint32_t wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t o = wave_or(orv[w]);
    uint64_t a = wave_and(andv[w]);
    if (lane_id() == 0) {
      s_red[(2 * w) * 4 + wave] = o;
      s_red[(2 * w + 1) * 4 + wave] = a;
    }
  }
  __syncthreads();
  if (threadIdx.x < (uint32_t)W) {
    const int w = threadIdx.x;
    uint64_t o = 0, a = ~0ull;
    for (int i = 0; i < kBlock / 64; ++i) {
      o |= s_red[(2 * w) * 4 + i];
      a &= s_red[(2 * w + 1) * 4 + i];
    }
    // OR only gains bits and AND only loses them, so a workgroup whose values
    // are already folded in (read back, possibly stale: a stale value has
    // fewer OR bits / more AND bits, which only causes an extra atomic)
    // skips its atomic; after the first few workgroups almost all do.
    const uint32_t r = epoch % kRing;
    const uint64_t co = ld_agent(reinterpret_cast<const uint64_t*>(&meta->or_mask[r][w]));
    const uint64_t ca = ld_agent(reinterpret_cast<const uint64_t*>(&meta->and_mask[r][w]));
    if ((co | o) != co) atomicOr(&meta->or_mask[r][w], (unsigned long long)o);
    if ((ca & a) != ca) atomicAnd(&meta->and_mask[r][w], (unsigned long long)a);
  }
}

}  // namespace sparqs
