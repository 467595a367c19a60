// gfx950 kernels of the sparse register-level simulator.
//
// State layout in HBM (structure of arrays): key word w of entry i at
// keys.w[w][i] (uint64), amplitude at amp[i] (double2 = re, im).  Register r
// occupies bits [off_r, off_r + width_r) of one key word; qubit q of r is bit
// off_r + q.
//
//  * k_perm     - a fused run of non-interference ops (X/CNOT/Toffoli, register
//                 add/sub, multiply by an odd constant, XOR, QRAM load/unload,
//                 the reflection R): every entry is updated in place while its
//                 key sits in registers (Sec. "Non-interference operations";
//                 QRAM equation; QLSS reflection R).
//  * k_sort_hist / k_sort_scan / k_sort_pass
//               - LSD radix sort over multi-word keys (one pass per 8-bit digit
//                 of the bits that vary): LDS digit histograms, wave64 ballot
//                 ranking, decoupled look-back for the global digit offsets,
//                 LDS-staged scatter.  It puts coherent branches (equal idle
//                 qubits) next to each other (Sec. "Interference operations",
//                 first step).
//  * k_group    - applies a branching op to each group of coherent branches
//                 (second step of the same section), creating up to 2^k
//                 children, merging contributions that land on the same key,
//                 and removing entries whose |a|^2 falls below eps^2 (the
//                 zero-clearing step), compacted with a look-back prefix.
//  * k_filter   - threshold prune / measurement collapse with compaction.
#include "kernels_common.hpp"

namespace sparqs {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ uint64_t sel_word(const uint64_t (&k)[W], uint32_t w) {
  uint64_t v = k[0];
#pragma unroll
  for (int i = 1; i < W; ++i)
    if (w == (uint32_t)i) v = k[i];
  return v;
}

template <int W>
__device__ __forceinline__ void put_word(uint64_t (&k)[W], uint32_t w, uint64_t v) {
#pragma unroll
  for (int i = 0; i < W; ++i)
    if (w == (uint32_t)i) k[i] = v;
}

template <int W>
__device__ __forceinline__ bool controls_hold(const uint64_t (&k)[W], const uint64_t* cmask,
                                              const uint64_t* cval) {
  bool on = true;
#pragma unroll
  for (int w = 0; w < W; ++w) on = on && ((k[w] & cmask[w]) == cval[w]);
  return on;
}

// Complex product with every product and sum rounded on its own:
// (a + ib)(c + id) = (ac - bd) + i(ad + bc).
__device__ __forceinline__ double2 cmul(double2 a, double cr, double ci) {
  double2 r;
  r.x = a.x * cr - a.y * ci;
  r.y = a.x * ci + a.y * cr;
  return r;
}

// Keep an amplitude unless |a|^2 < eps^2 or it is exactly zero.  The product
// and sum are rounded separately (the file is built without contraction).
__device__ __forceinline__ bool keep_amp(double re, double im, double eps2) {
  const double n2 = re * re + im * im;
  return !(n2 < eps2) && !(re == 0.0 && im == 0.0);
}

// ---------------------------------------------------------------------------
// k_perm: fused run of non-branching ops
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void perm_apply(uint64_t (&k)[W], double2& a, const PermOp& op) {
  if (op.nctl_words && !controls_hold<W>(k, op.cmask, op.cval)) return;
  const uint64_t dw = sel_word<W>(k, op.dst_word);
  const uint64_t dv = (dw >> op.dst_shift) & op.dst_mask;
  uint64_t nv;
  switch (op.kind) {
    case PK_XMASK:
    case PK_XORC:
      nv = dv ^ op.imm;
      break;
    case PK_ADD:
      nv = (dv + ((sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask)) & op.dst_mask;
      break;
    case PK_SUB:
      nv = (dv - ((sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask)) & op.dst_mask;
      break;
    case PK_MULC:
      nv = (dv * op.imm) & op.dst_mask;
      break;
    case PK_XOR:
      nv = (dv ^ ((sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask)) & op.dst_mask;
      break;
    case PK_QRAM: {
      const uint64_t addr = (sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask;
      const uint64_t t = op.table_words32 ? (uint64_t)((const uint32_t*)op.table)[addr]
                                          : ((const uint64_t*)op.table)[addr];
      nv = (dv ^ t) & op.dst_mask;
      break;
    }
    case PK_REFLECT0: {
      // R = i(2|0><0| - I): +i on a zero field, -i otherwise (exact)
      const double re = a.x, im = a.y;
      if (dv == 0) {
        a.x = -im;
        a.y = re;
      } else {
        a.x = im;
        a.y = -re;
      }
      return;
    }
    case PK_DIAG:
    case PK_ADIAG: {
      // one qubit at a time, ascending: the factor of the matrix element
      // that takes this qubit's bit to its output bit
      for (uint64_t m = op.imm; m; m &= m - 1) {
        const uint32_t b = (uint32_t)((dw >> __builtin_ctzll(m)) & 1ull);
        a = cmul(a, op.fac[b][0], op.fac[b][1]);
      }
      if (op.kind == PK_ADIAG) put_word<W>(k, op.dst_word, dw ^ op.imm);
      return;
    }
    case PK_ADDC:
      nv = (dv + op.imm) & op.dst_mask;
      break;
    case PK_MUL: {
      const uint64_t x = (sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask;
      const uint64_t y = (sel_word<W>(k, op.src2_word) >> op.src2_shift) & op.src2_mask;
      nv = (dv ^ (x * y)) & op.dst_mask;
      break;
    }
    case PK_DIV: {
      const uint64_t x = (sel_word<W>(k, op.src_word) >> op.src_shift) & op.src_mask;
      const uint64_t y = (sel_word<W>(k, op.src2_word) >> op.src2_shift) & op.src2_mask;
      const uint64_t q = y ? x / y : ~0ull, r = y ? x % y : x;
      // remainder register first (it never overlaps the quotient's)
      const uint64_t w2 = sel_word<W>(k, op.dst2_word);
      const uint64_t m2 = op.dst2_mask << op.dst2_shift;
      const uint64_t r2 = (((w2 >> op.dst2_shift) & op.dst2_mask) ^ r) & op.dst2_mask;
      put_word<W>(k, op.dst2_word, (w2 & ~m2) | (r2 << op.dst2_shift));
      const uint64_t dw2 = sel_word<W>(k, op.dst_word);
      const uint64_t mq = op.dst_mask << op.dst_shift;
      put_word<W>(k, op.dst_word, (dw2 & ~mq) | ((((dv ^ q) & op.dst_mask) << op.dst_shift) & mq));
      return;
    }
    default:
      return;
  }
  const uint64_t m = op.dst_mask << op.dst_shift;
  put_word<W>(k, op.dst_word, (dw & ~m) | ((nv << op.dst_shift) & m));
}

template <int W, bool AMP>
__global__ __launch_bounds__(kBlock) void k_perm(KeyPtrs<W> keys, double2* __restrict__ amp,
                                                 uint32_t ns, const PermOp* __restrict__ ops,
                                                 uint32_t nops, uint32_t write_words,
                                                 DevMeta* meta, uint32_t epoch) {
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  if (launch_prologue(meta, epoch)) return;
  const uint64_t n = meta->nring[ns & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) meta->upd += n * nops;
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    uint64_t k[W];
#pragma unroll
    for (int w = 0; w < W; ++w) k[w] = keys.w[w][i];
    double2 a = make_double2(0.0, 0.0);
    if (AMP) a = amp[i];
    for (uint32_t o = 0; o < nops; ++o) perm_apply<W>(k, a, ops[o]);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (write_words & (1u << w)) keys.w[w][i] = k[w];
      orv[w] |= k[w];
      andv[w] &= k[w];
    }
    if (AMP) amp[i] = a;
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// k_perm_fast: the same ops in 32-bit form for keys of 1 or 2 words.  One
// switch case per (kind, half indices), so every case is straight-line code
// on named registers; each thread carries E entries so the per-op decode is
// shared.  Op records are read with scalar loads, the next one while the
// current op runs, so a record's fields are scalar operands and the decode
// waits on no memory round trip.
// ---------------------------------------------------------------------------
namespace fast {

// X / XORC on one half: h ^= imm
template <int T, int E>
__device__ __forceinline__ void xm(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) h[j][T] ^= op.imm;
}

// one control: bit cb of half C taken as 0 / all ones (signed one-bit
// extract), inverted when the required value is 0
template <int T, int C, bool NEG, int E>
__device__ __forceinline__ void xc1(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)h[j][C], op.a, 1u);
    h[j][T] ^= op.imm & (NEG ? ~m : m);
  }
}

// two controls; cvm / cvm2 are all ones where the required value is 0
template <int T, int C, int C2, int E>
__device__ __forceinline__ void xc2(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)h[j][C], op.a, 1u) ^ op.c;
    const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int)h[j][C2], op.b, 1u) ^ op.d;
    h[j][T] ^= op.imm & m1 & m2;
  }
}

// whole halves: h[D] (+|-|^)= h[S]
enum { OP_ADD, OP_SUB, OP_XOR };
template <int K, int D, int S, int E>
__device__ __forceinline__ void whole(uint32_t (&h)[E][4]) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if (K == OP_ADD) h[j][D] += h[j][S];
    else if (K == OP_SUB) h[j][D] -= h[j][S];
    else h[j][D] ^= h[j][S];
  }
}

// fields: the source's low sw bits (sw = min(source width, destination
// width) < 32: only those reach the result modulo 2^width) are shifted to
// the destination's place and combined there; carries and borrows run only
// upwards, so bits outside the destination field are restored by the mask
template <int K, int D, int S, int E>
__device__ __forceinline__ void field(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t v = __builtin_amdgcn_ubfe(h[j][S], op.c, op.d) << op.a;
    const uint32_t x = h[j][D];
    if (K == OP_ADD) h[j][D] = ((x + v) & op.b) | (x & ~op.b);
    else if (K == OP_SUB) h[j][D] = ((x - v) & op.b) | (x & ~op.b);
    else h[j][D] = x ^ v;
  }
}

template <int D, int E>
__device__ __forceinline__ void mul_whole(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) h[j][D] *= op.imm;
}

// field times an odd constant modulo 2^width (width < 32)
template <int D, int E>
__device__ __forceinline__ void mul_field(uint32_t (&h)[E][4], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t v = (__builtin_amdgcn_ubfe(h[j][D], op.a, op.d) * op.imm) << op.a;
    h[j][D] = (v & op.b) | (h[j][D] & ~op.b);
  }
}

// data field ^= table32[address field]
template <int D, int S, int E>
__device__ __forceinline__ void qram(uint32_t (&h)[E][4], const FastOp& op) {
  const uint32_t* table = reinterpret_cast<const uint32_t*>(((uint64_t)op.f << 32) | op.e);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t t = table[(h[j][S] >> op.c) & op.d];
    h[j][D] ^= (t << op.a) & op.b;
  }
}

// amplitude times +i where the field is 0, -i elsewhere
template <int D, int E>
__device__ __forceinline__ void refl(const uint32_t (&h)[E][4], double2 (&a)[E], const FastOp& op) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const double re = a[j].x, im = a[j].y;
    if ((h[j][D] & op.b) == 0u) {
      a[j].x = -im;
      a[j].y = re;
    } else {
      a[j].x = im;
      a[j].y = -re;
    }
  }
}

template <int W, int E>
__device__ __forceinline__ void gen(uint32_t (&h)[E][4], double2 (&a)[E], const PermOp& g) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    uint64_t k[W];
#pragma unroll
    for (int w = 0; w < W; ++w) k[w] = (uint64_t)h[j][2 * w] | ((uint64_t)h[j][2 * w + 1] << 32);
    perm_apply<W>(k, a[j], g);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      h[j][2 * w] = (uint32_t)k[w];
      h[j][2 * w + 1] = (uint32_t)(k[w] >> 32);
    }
  }
}

}  // namespace fast

// case lists: one case per half (index x), per (target, control) pair
// (t*4 + c), per (target, control, control) triple
#define SQ_C4(M, B) M(B, 0) M(B, 1) M(B, 2) M(B, 3)
#define SQ_C16(M, B) SQ_C4(M, B) SQ_C4(M, B + 4) SQ_C4(M, B + 8) SQ_C4(M, B + 12)
#define SQ_C64(M, B) SQ_C16(M, B) SQ_C16(M, B + 16) SQ_C16(M, B + 32) SQ_C16(M, B + 48)
#define SQ_XM(B, x) case (B) + (x): fast::xm<x, E>(h, op); break;
#define SQ_XC1(B, x) case (B) + (x): fast::xc1<(((B) + (x) - F_XC1) >> 2) & 3, ((B) + (x) - F_XC1) & 3, false, E>(h, op); break;
#define SQ_XC1N(B, x) case (B) + (x): fast::xc1<(((B) + (x) - F_XC1N) >> 2) & 3, ((B) + (x) - F_XC1N) & 3, true, E>(h, op); break;
#define SQ_XC2(B, x) case (B) + (x): fast::xc2<(((B) + (x) - F_XC2) >> 4) & 3, (((B) + (x) - F_XC2) >> 2) & 3, ((B) + (x) - F_XC2) & 3, E>(h, op); break;
#define SQ_WH(B, x, K, F0) case (B) + (x): fast::whole<K, (((B) + (x) - F0) >> 2) & 3, ((B) + (x) - F0) & 3, E>(h); break;
#define SQ_FI(B, x, K, F0) case (B) + (x): fast::field<K, (((B) + (x) - F0) >> 2) & 3, ((B) + (x) - F0) & 3, E>(h, op); break;
#define SQ_ADDA(B, x) SQ_WH(B, x, fast::OP_ADD, F_ADDA)
#define SQ_SUBA(B, x) SQ_WH(B, x, fast::OP_SUB, F_SUBA)
#define SQ_XORA(B, x) SQ_WH(B, x, fast::OP_XOR, F_XORA)
#define SQ_ADDF(B, x) SQ_FI(B, x, fast::OP_ADD, F_ADDF)
#define SQ_SUBF(B, x) SQ_FI(B, x, fast::OP_SUB, F_SUBF)
#define SQ_XORF(B, x) SQ_FI(B, x, fast::OP_XOR, F_XORF)
#define SQ_MULA(B, x) case (B) + (x): fast::mul_whole<x, E>(h, op); break;
#define SQ_MULF(B, x) case (B) + (x): fast::mul_field<x, E>(h, op); break;
#define SQ_QRAM(B, x) case (B) + (x): fast::qram<(((B) + (x) - F_QRAM) >> 2) & 3, ((B) + (x) - F_QRAM) & 3, E>(h, op); break;
#define SQ_REFL(B, x) case (B) + (x): fast::refl<x, E>(h, a, op); break;

template <int W, int E, bool AMP>
__device__ __forceinline__ void fast_step(uint32_t (&h)[E][4], double2 (&a)[E], const FastOp& op,
                                          const PermOp* __restrict__ gops) {
  switch (op.code) {
    SQ_C4(SQ_XM, F_XM)
    SQ_C16(SQ_XC1, F_XC1)
    SQ_C16(SQ_XC1N, F_XC1N)
    SQ_C64(SQ_XC2, F_XC2)
    SQ_C16(SQ_ADDA, F_ADDA)
    SQ_C16(SQ_ADDF, F_ADDF)
    SQ_C16(SQ_SUBA, F_SUBA)
    SQ_C16(SQ_SUBF, F_SUBF)
    SQ_C16(SQ_XORA, F_XORA)
    SQ_C16(SQ_XORF, F_XORF)
    SQ_C4(SQ_MULA, F_MULA)
    SQ_C4(SQ_MULF, F_MULF)
    SQ_C16(SQ_QRAM, F_QRAM)
    case F_REFL + 0: if (AMP) fast::refl<0, E>(h, a, op); break;
    case F_REFL + 1: if (AMP) fast::refl<1, E>(h, a, op); break;
    case F_REFL + 2: if (AMP) fast::refl<2, E>(h, a, op); break;
    case F_REFL + 3: if (AMP) fast::refl<3, E>(h, a, op); break;
    case F_GEN: fast::gen<W, E>(h, a, gops[op.e]); break;
    default: break;
  }
}
#undef SQ_C4
#undef SQ_C16
#undef SQ_C64
#undef SQ_XM
#undef SQ_XC1
#undef SQ_XC1N
#undef SQ_XC2
#undef SQ_WH
#undef SQ_FI
#undef SQ_ADDA
#undef SQ_SUBA
#undef SQ_XORA
#undef SQ_ADDF
#undef SQ_SUBF
#undef SQ_XORF
#undef SQ_MULA
#undef SQ_MULF
#undef SQ_QRAM
#undef SQ_REFL

// A run of non-branching ops on E entries per thread.  The record of op o+1
// is loaded (scalar load) after op o's fields have arrived and before op o
// runs, so its latency hides behind op o; the empty asm statement with a
// memory clobber keeps the compiler from hoisting that load above the wait
// for op o's record (the scalar counter cannot wait for one of two loads).
// Two record registers alternate (the loop is unrolled twice), so no record
// is copied between them.  The records are followed by one padding record,
// which the last prefetch reads.  They are read through the constant address
// space (they do not change during a launch), which makes every such read a
// scalar load whatever else the kernel stores.
__device__ __forceinline__ FastOp load_rec(const FastOp* p) {
  typedef const __attribute__((address_space(4))) uint32_t ConstU32;
  ConstU32* q = (ConstU32*)p;
  FastOp r;
  r.code = q[0];
  r.imm = q[1];
  r.a = q[2];
  r.b = q[3];
  r.c = q[4];
  r.d = q[5];
  r.e = q[6];
  r.f = q[7];
  return r;
}

template <int W, int E, bool AMP>
__device__ __forceinline__ void run_ops(uint32_t (&h)[E][4], double2 (&a)[E], const FastOp* __restrict__ ops,
                                        uint32_t nops, const PermOp* __restrict__ gops) {
  if (nops == 0) return;
  const FastOp* p = ops;
  const FastOp* const last = ops + (nops - 1);
  FastOp r0 = load_rec(p);
  for (;;) {
    asm volatile("" ::"s"(r0.code) : "memory");
    const FastOp r1 = load_rec(p + 1);
    fast_step<W, E, AMP>(h, a, r0, gops);
    if (p == last) break;
    asm volatile("" ::"s"(r1.code) : "memory");
    r0 = load_rec(p + 2);
    fast_step<W, E, AMP>(h, a, r1, gops);
    if (p + 1 == last) break;
    p += 2;
  }
}

template <int W, int E, bool AMP>
__global__ __launch_bounds__(kBlock) void k_perm_fast(KeyPtrs<W> keys, double2* __restrict__ amp, uint32_t ns,
                                                      const FastOp* __restrict__ ops, uint32_t nops,
                                                      const PermOp* __restrict__ gops, uint32_t write_words,
                                                      DevMeta* meta, uint32_t epoch) {
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  if (launch_prologue(meta, epoch)) return;
  const uint64_t n = meta->nring[ns & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    meta->upd += n * nops;
    if ((uint64_t)gridDim.x * kBlock * E < n) raise_error(meta, kErrGrid, epoch);
  }
  // the grid comes from an upper bound of the count
  if ((uint64_t)blockIdx.x * kBlock * E >= n) return;
  uint32_t h[E][4];
  double2 a[E];
  const uint64_t base = (uint64_t)blockIdx.x * kBlock * E + threadIdx.x;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    h[j][2] = h[j][3] = 0u;
    a[j] = make_double2(0.0, 0.0);
    if (i < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t v = keys.w[w][i];
        h[j][2 * w] = (uint32_t)v;
        h[j][2 * w + 1] = (uint32_t)(v >> 32);
      }
      if (AMP) a[j] = amp[i];
    } else {
      h[j][0] = h[j][1] = 0u;
    }
  }
  run_ops<W, E, AMP>(h, a, ops, nops, gops);
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    if (i >= n) continue;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t v = (uint64_t)h[j][2 * w] | ((uint64_t)h[j][2 * w + 1] << 32);
      if (write_words & (1u << w)) keys.w[w][i] = v;
      orv[w] |= v;
      andv[w] &= v;
    }
    if (AMP) amp[i] = a[j];
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ uint32_t digit_of(const uint64_t (&k)[W], const PassDesc& pd) {
  uint32_t d = 0;
  for (uint32_t j = 0; j < pd.nf; ++j) {
    const uint32_t f = pd.f[j];
    const uint32_t word = f & 3u, shift = (f >> 2) & 63u, width = (f >> 8) & 15u,
                   ds = (f >> 12) & 15u;
    const uint64_t v = sel_word<W>(k, word);
    d |= (uint32_t)((v >> shift) & ((1ull << width) - 1ull)) << ds;
  }
  return d;
}

// Per-workgroup digit histograms of every pass in one read of the keys.  Each
// workgroup takes a contiguous chunk, U entries per thread per step with the
// loads issued together; for each pass its field descriptors are read once
// per step (into scalar registers) and applied to the U entries.  Keys are
// often nearly sorted, so a wave whose lanes all carry the same digit adds
// its count with one LDS atomic.
template <int W>
__global__ __launch_bounds__(kBlock) void k_sort_hist(KeyPtrs<W> keys, uint32_t ns, const DevMeta* meta,
                                                      SortPlan plan, unsigned long long* __restrict__ ghist) {
  constexpr int U = W <= 2 ? 8 : 4;
  extern __shared__ uint32_t s_h[];  // npass * 256
  const uint32_t np = plan.npass;
  // the entry count of slot ns (the grid comes from an upper bound; workgroups
  // past the count add nothing), on the view [base, n) of batched rounds
  const uint64_t vb = meta->base;
  const uint64_t n = meta->nring[ns & 1] - vb;
  offset_keys<W>(keys, vb);
  for (uint32_t i = threadIdx.x; i < np * kRadix; i += kBlock) s_h[i] = 0;
  __syncthreads();
  const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < n ? lo + chunk : n;
  // software pipelined: the next step's keys are loaded before this step's
  // digits are counted
  uint64_t kn[U][W];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t i = lo + (uint64_t)u * kBlock + threadIdx.x;
#pragma unroll
    for (int w = 0; w < W; ++w) kn[u][w] = i < hi ? keys.w[w][i] : 0ull;
  }
  for (uint64_t base = lo; base < hi; base += (uint64_t)kBlock * U) {
    uint64_t k[U][W];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * kBlock + threadIdx.x;
      valid[u] = i < hi;
#pragma unroll
      for (int w = 0; w < W; ++w) k[u][w] = kn[u][w];
    }
    const uint64_t nb = base + (uint64_t)kBlock * U;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = nb + (uint64_t)u * kBlock + threadIdx.x;
#pragma unroll
      for (int w = 0; w < W; ++w) kn[u][w] = i < hi ? keys.w[w][i] : 0ull;
    }
    for (uint32_t p = 0; p < np; ++p) {
      const uint32_t nf = plan.pass[p].nf;
      uint32_t fw[kMaxFields];
#pragma unroll
      for (int j = 0; j < kMaxFields; ++j) fw[j] = (uint32_t)j < nf ? plan.pass[p].f[j] : 0u;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t active = __ballot(valid[u]);
        if (!valid[u]) continue;
        uint32_t d = 0;
#pragma unroll
        for (int j = 0; j < kMaxFields; ++j) {
          if ((uint32_t)j >= nf) break;
          const uint32_t f = fw[j];
          const uint32_t word = f & 3u, shift = (f >> 2) & 63u, width = (f >> 8) & 15u, ds = (f >> 12) & 15u;
          d |= (uint32_t)((sel_word<W>(k[u], word) >> shift) & ((1ull << width) - 1ull)) << ds;
        }
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        if (__ballot(d == d0) == active) {
          if (lane_id() == (uint32_t)__builtin_ctzll(active)) atomicAdd(&s_h[p * kRadix + d0], (uint32_t)__popcll(active));
        } else {
          atomicAdd(&s_h[p * kRadix + d], 1u);
        }
      }
    }
  }
  __syncthreads();
  // fold the workgroup's counts into the global histograms (zeroed before
  // the launch); integer sums, so the order of the atomics does not matter
  for (uint32_t i = threadIdx.x; i < np * kRadix; i += kBlock)
    if (s_h[i]) atomicAdd(&ghist[i], (unsigned long long)s_h[i]);
}

// Scan the digit counts of pass blockIdx.x into the first global position of
// every digit.
static __global__ __launch_bounds__(kBlock) void k_sort_scan(const unsigned long long* __restrict__ ghist,
                                                      uint64_t* __restrict__ digit_start) {
  __shared__ uint64_t s_tmp[4];
  const uint32_t p = blockIdx.x, d = threadIdx.x;
  const uint64_t c = ghist[p * kRadix + d];
  uint64_t tot;
  const uint64_t ex = block_excl_scan<uint64_t>(c, s_tmp, tot);
  digit_start[p * kRadix + d] = ex;
}

// One LSD pass: stable scatter of (keys, amplitude) by the digit `pd`.
template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_sort_pass(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                      KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                      uint32_t ns, PassDesc pd,
                                                      const uint64_t* __restrict__ digit_start,
                                                      uint64_t* lb, DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr int TILE = kBlock * ITEMS;
  __shared__ uint32_t s_wcount[kBlock / 64][kRadix];
  __shared__ uint32_t s_toff[kRadix];
  __shared__ uint64_t s_gbase[kRadix];
  __shared__ uint8_t s_digit[TILE];
  __shared__ __align__(16) uint64_t s_stage[TILE];
  __shared__ uint64_t s_scan[4];
  __shared__ uint32_t s_tile;

  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // The count is read on the device (a sort does not change it) and the grid
  // comes from an upper bound: workgroups past the count's tiles leave before
  // taking a tile ticket, so the tickets cover exactly the count's tiles.
  // Batched rounds sort the view [base, n).  Both come with the prologue's
  // round trip.
  PrologueReads pr;
  if (launch_prologue_reads(meta, epoch, ns, true, nullptr, &pr)) return;
  const uint64_t vb = pr.base;
  const uint64_t n = pr.n - vb;
  offset_keys<W>(in_keys, vb);
  offset_keys<W>(out_keys, vb);
  in_amp += vb;
  out_amp += vb;
  if (blockIdx.x == 0 && tid == 0 && (uint64_t)gridDim.x * TILE < n) raise_error(meta, kErrGrid, epoch);
  // xo == 2: tickets in chunks per XCD (every workgroup takes one)
  if (xo != 2 && (uint64_t)blockIdx.x * TILE >= n) return;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) s_wcount[w][tid] = 0;
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  if (tile_out_of_range(tile, (n + TILE - 1) / TILE, &meta->err, xo)) return;
  const uint64_t base = (uint64_t)tile * TILE;
  const uint32_t tile_n = (uint32_t)min((uint64_t)TILE, n - base);

  uint64_t k[ITEMS][W];
  uint32_t dig[ITEMS], rank[ITEMS];
  // all key loads first (the digit extraction loops would otherwise make
  // each load wait for the previous item)
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
#pragma unroll
    for (int w = 0; w < W; ++w) k[i][w] = le < tile_n ? in_keys.w[w][base + le] : 0ull;
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
    dig[i] = le < tile_n ? digit_of<W>(k[i], pd) : 0u;
  }
  // stable rank within the wave's chunk: ballot-match on the digit bits
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
    const bool valid = le < tile_n;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (dig[i] >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t below = mbcnt(m);
    uint32_t prior = 0;
    if (valid) prior = s_wcount[wave][dig[i]];
    rank[i] = prior + below;
    if (valid && below == 0) s_wcount[wave][dig[i]] = prior + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // per digit: exclusive offsets across waves, tile count, look-back
  uint32_t cnt;
  {
    const uint32_t c0 = s_wcount[0][tid], c1 = s_wcount[1][tid], c2 = s_wcount[2][tid],
                   c3 = s_wcount[3][tid];
    s_wcount[0][tid] = 0;
    s_wcount[1][tid] = c0;
    s_wcount[2][tid] = c0 + c1;
    s_wcount[3][tid] = c0 + c1 + c2;
    cnt = c0 + c1 + c2 + c3;
  }
  const uint64_t prev = lookback_digit(lb, tile, tid, cnt, epoch, &meta->err);
  uint64_t tot;
  const uint64_t loc = block_excl_scan<uint64_t>((uint64_t)cnt, s_scan, tot);
  s_toff[tid] = (uint32_t)loc;
  s_gbase[tid] = digit_start[tid] + prev - loc;
  __syncthreads();
  uint32_t pos[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
    if (le < tile_n) {
      pos[i] = s_toff[dig[i]] + s_wcount[wave][dig[i]] + rank[i];
      s_digit[pos[i]] = (uint8_t)dig[i];
    }
  }
  // scatter one 8-byte column at a time through LDS
#pragma unroll
  for (int w = 0; w < W; ++w) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
      if (le < tile_n) s_stage[pos[i]] = k[i][w];
    }
    __syncthreads();
    for (uint32_t j = tid; j < tile_n; j += kBlock) {
      const uint64_t dst = s_gbase[s_digit[j]] + j;
      if (dst < n) out_keys.w[w][dst] = s_stage[j];
    }
    __syncthreads();
  }
  double2 av[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
    av[i] = le < tile_n ? in_amp[base + le] : make_double2(0.0, 0.0);
  }
  // Amplitudes go out as whole 16-byte values (two 8-byte passes would write
  // every output line in two halves at different times), staged half a tile
  // at a time in the same LDS.
  double2* s_amp = reinterpret_cast<double2*>(s_stage);
  constexpr uint32_t HALF = TILE / 2;
#pragma unroll
  for (uint32_t h0 = 0; h0 < (uint32_t)TILE; h0 += HALF) {
    if (h0) __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t le = wave * (ITEMS * 64) + i * 64 + lane;
      if (le < tile_n && pos[i] >= h0 && pos[i] < h0 + HALF) s_amp[pos[i] - h0] = av[i];
    }
    __syncthreads();
    const uint32_t hn = tile_n > h0 ? min(HALF, tile_n - h0) : 0u;
    for (uint32_t j = tid; j < hn; j += kBlock) {
      const uint64_t dst = s_gbase[s_digit[h0 + j]] + h0 + j;
      if (dst < n) out_amp[dst] = s_amp[j];
    }
  }
}

// ---------------------------------------------------------------------------
// k_group: apply a branching op to groups of coherent branches
// ---------------------------------------------------------------------------
// MODE_GROUP: members of a group (equal key outside the target bits) are
// contiguous; the first member leads.  MODE_EXPAND: every entry is its own
// group (no target bit varies over the state).
enum { MODE_GROUP = 0, MODE_EXPAND = 1 };

template <int W>
__device__ __forceinline__ bool same_idle(const uint64_t (&a)[W], const uint64_t (&b)[W],
                                          const uint64_t* tmask) {
  bool eq = true;
#pragma unroll
  for (int w = 0; w < W; ++w) eq = eq && (((a[w] ^ b[w]) & ~tmask[w]) == 0);
  return eq;
}

template <int W, int K>
__device__ __forceinline__ uint32_t target_value(const uint64_t (&k)[W], const GroupOp& op) {
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) s |= (uint32_t)((sel_word<W>(k, op.tword[j]) >> op.tbit[j]) & 1ull) << j;
  return s;
}

template <int W, int K>
__device__ __forceinline__ void with_target_value(uint64_t (&k)[W], const GroupOp& op, uint32_t s) {
#pragma unroll
  for (int w = 0; w < W; ++w) k[w] &= ~op.tmask[w];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if ((s >> j) & 1u) {
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (op.tword[j] == (uint32_t)w) k[w] |= 1ull << op.tbit[j];
    }
  }
}

// Offsets of ITEMS counts per thread in element order (item-major, then
// thread): ITEMS wave scans and one barrier.  Returns the tile total.
template <int ITEMS>
__device__ __forceinline__ uint64_t tile_offsets(const uint32_t (&cnt)[ITEMS], uint32_t (&off)[ITEMS],
                                                 uint32_t (*s_wtot)[kBlock / 64]) {
  const uint32_t wave = threadIdx.x >> 6, lane = lane_id();
  uint32_t inc[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    inc[i] = wave_incl_scan<uint32_t>(cnt[i]);
    if (lane == 63) s_wtot[i][wave] = inc[i];
  }
  __syncthreads();
  uint64_t run = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    uint32_t pre = 0, row = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBlock / 64; ++w) {
      const uint32_t x = s_wtot[i][w];
      if (w < wave) pre += x;
      row += x;
    }
    off[i] = (uint32_t)run + pre + inc[i] - cnt[i];
    run += row;
  }
  return run;
}

template <int W, int K, int MODE, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_group(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                  KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                  uint32_t ns, uint64_t cap, GroupOp op, uint64_t* lb,
                                                  DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr uint32_t G = 1u << K;
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  uint64_t n;
  if (!emit_begin(meta, ns, epoch, TILE, &n, xo)) return;
  if (op.upd && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&meta->upd, (unsigned long long)(n * op.upd));
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;

  uint64_t key[ITEMS][W];
  double2 v[ITEMS][G];
  uint32_t keepm[ITEMS], cnt[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = (uint64_t)tile * TILE + (uint64_t)it * kBlock + threadIdx.x;
    uint32_t present = 0;
#pragma unroll
    for (uint32_t s = 0; s < G; ++s) v[it][s] = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < W; ++w) key[it][w] = 0;
    bool lead = false;
    if (e < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) key[it][w] = in_keys.w[w][e];
      lead = true;
      if (MODE == MODE_GROUP && e > 0) {
        uint64_t prv[W];
#pragma unroll
        for (int w = 0; w < W; ++w) prv[w] = in_keys.w[w][e - 1];
        lead = !same_idle<W>(key[it], prv, op.tmask);
      }
    }
    if (lead) {
      const bool ctl = !op.has_ctl || controls_hold<W>(key[it], op.cmask, op.cval);
      const uint32_t s0 = target_value<W, K>(key[it], op);
      const double2 a0 = in_amp[e];
#pragma unroll
      for (uint32_t t = 0; t < G; ++t)
        if (t == s0) v[it][t] = a0;
      present = 1u << s0;
      if (MODE == MODE_GROUP) {
        for (uint32_t j = 1; j < G && e + j < n; ++j) {
          uint64_t nk[W];
#pragma unroll
          for (int w = 0; w < W; ++w) nk[w] = in_keys.w[w][e + j];
          if (!same_idle<W>(key[it], nk, op.tmask)) break;
          const uint32_t s = target_value<W, K>(nk, op);
          if (present & (1u << s)) atomicOr(&meta->err, kErrGroup);
          const double2 a = in_amp[e + j];
#pragma unroll
          for (uint32_t t = 0; t < G; ++t)
            if (t == s) v[it][t] = a;
          present |= 1u << s;
        }
      }
      if (ctl) {
        // one butterfly stage per target qubit, ascending; a child exists when
        // some present parent reaches it through a nonzero matrix element
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
          for (uint32_t s = 0; s < G; ++s) {
            if ((s >> j) & 1u) continue;
            const uint32_t s1 = s | (1u << j);
            const double2 a0 = v[it][s], a1 = v[it][s1];
            const bool p0 = (present >> s) & 1u, p1 = (present >> s1) & 1u;
            double2 b0, b1;
            b0.x = op.m[0][0] * a0.x + op.m[0][1] * a1.x;
            b0.y = op.m[0][0] * a0.y + op.m[0][1] * a1.y;
            b1.x = op.m[1][0] * a0.x + op.m[1][1] * a1.x;
            b1.y = op.m[1][0] * a0.y + op.m[1][1] * a1.y;
            const bool q0 = (p0 && op.m[0][0] != 0.0) || (p1 && op.m[0][1] != 0.0);
            const bool q1 = (p0 && op.m[1][0] != 0.0) || (p1 && op.m[1][1] != 0.0);
            v[it][s] = b0;
            v[it][s1] = b1;
            present = (present & ~((1u << s) | (1u << s1))) | ((uint32_t)q0 << s) | ((uint32_t)q1 << s1);
          }
        }
      }
    }
    keepm[it] = 0;
    if (lead) {
#pragma unroll
      for (uint32_t s = 0; s < G; ++s)
        if (((present >> s) & 1u) && keep_amp(v[it][s].x, v[it][s].y, op.eps2)) keepm[it] |= 1u << s;
    }
    cnt[it] = (uint32_t)__popc(keepm[it]);
  }
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = ex + tile_total;
        if (ex + tile_total > cap) raise_error(meta, kErrCapacity, epoch);
        else atomicMax(&meta->peak, (unsigned long long)(ex + tile_total));
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    uint64_t p = s_off + off[it];
    if (!keepm[it]) continue;
#pragma unroll
    for (uint32_t s = 0; s < G; ++s) {
      if (!((keepm[it] >> s) & 1u)) continue;
      uint64_t ok[W];
#pragma unroll
      for (int w = 0; w < W; ++w) ok[w] = key[it][w];
      with_target_value<W, K>(ok, op, s);
      if (p < cap) {
#pragma unroll
        for (int w = 0; w < W; ++w) out_keys.w[w][p] = ok[w];
        out_amp[p] = v[it][s];
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        orv[w] |= ok[w];
        andv[w] &= ok[w];
      }
      ++p;
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// k_expand_slots: expand mode on K >= 2 targets (every entry alone in its
// group), one thread per (entry, child) slot: slot q is child c = q mod 2^K of
// entry q / 2^K, so consecutive lanes write consecutive outputs.  With the
// entry's target value s0, child c gets a0 * m[c_0][s0_0] * ... * m[c_K-1][s0_K-1]
// (real factors taken in ascending j, as the butterfly stages of k_group
// would, so the two agree bit for bit) and exists when every factor is
// nonzero; where the controls fail only c = s0 exists (the entry passes
// through).  Kept children are compacted (tile scan and look-back over slots).
// ---------------------------------------------------------------------------
template <int W, int K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_expand_slots(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                         KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                         uint32_t ns, uint64_t cap, GroupOp op, uint64_t* lb,
                                                         DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr uint32_t G = 1u << K;
  constexpr uint32_t TILE = kBlock * ITEMS;     // slots per tile
  static_assert(TILE % G == 0, "a tile holds whole entries");
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  uint64_t n;
  if (!emit_begin(meta, ns, epoch, TILE / G, &n, xo)) return;
  if (op.upd && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&meta->upd, (unsigned long long)(n * op.upd));
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n * G + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;
  uint64_t key[ITEMS][W];
  double2 v[ITEMS];
  uint32_t cnt[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t q = (uint64_t)tile * TILE + (uint64_t)it * kBlock + threadIdx.x;
    const uint64_t e = q >> K;
    const uint32_t c = (uint32_t)q & (G - 1u);
    cnt[it] = 0;
    v[it] = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < W; ++w) key[it][w] = 0;
    if (e < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) key[it][w] = in_keys.w[w][e];
      const double2 a0 = in_amp[e];
      const uint32_t s0 = target_value<W, K>(key[it], op);
      const bool ctl = !op.has_ctl || controls_hold<W>(key[it], op.cmask, op.cval);
      bool exists;
      if (ctl) {
        double2 x = a0;
        exists = true;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const uint32_t cj = (c >> j) & 1u, sj = (s0 >> j) & 1u;
          const double f = cj ? (sj ? op.m[1][1] : op.m[1][0]) : (sj ? op.m[0][1] : op.m[0][0]);
          x.x = f * x.x;
          x.y = f * x.y;
          exists = exists && f != 0.0;
        }
        v[it] = x;
      } else {
        exists = c == s0;
        v[it] = a0;
      }
      with_target_value<W, K>(key[it], op, c);
      cnt[it] = (exists && keep_amp(v[it].x, v[it].y, op.eps2)) ? 1u : 0u;
    }
  }
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = ex + tile_total;
        if (ex + tile_total > cap) raise_error(meta, kErrCapacity, epoch);
        else atomicMax(&meta->peak, (unsigned long long)(ex + tile_total));
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (!cnt[it]) continue;
    const uint64_t p = s_off + off[it];
    if (p < cap) {
#pragma unroll
      for (int w = 0; w < W; ++w) out_keys.w[w][p] = key[it][w];
      out_amp[p] = v[it];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      orv[w] |= key[it][w];
      andv[w] &= key[it][w];
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// k_pair: a branching op on one target qubit, one thread per entry.  In a
// full pair (the two members adjacent, in either order) each member writes the
// child with its own target value; a member without partner writes both children;
// where the controls fail the entry passes through.  Children of one group
// stay adjacent, in target-value order, and every child is computed with the
// same expression as in k_group (m[r][0] * a0 + m[r][1] * a1, absent = 0).
// ---------------------------------------------------------------------------
// The children of the ITEMS entries e0 + it * kBlock + threadIdx.x of one
// tile: keep mask (bit r: child with target value r) and amplitudes.  Every
// thread of the workgroup calls it (group mode stages the tile in LDS).
// The value held by lane t ^ 1 (the other lane of the pair): a DPP quad
// permutation [1, 0, 3, 2] on each 32-bit half, no LDS traffic.
__device__ __forceinline__ uint64_t lane_pair_swap(uint64_t x) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), 0xB1, 0xF, 0xF, false);
  return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
}

template <int W, int MODE, int ITEMS, int NB = 0>
__device__ __forceinline__ bool pair_tile(const KeyPtrs<W>& in_keys, const double2* __restrict__ in_amp,
                                          uint64_t n, uint64_t e0, const GroupOp& op, uint64_t* s_stage,
                                          uint64_t (&key)[ITEMS][W], double2 (&out)[ITEMS][2],
                                          uint32_t (&keepm)[ITEMS]) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  const uint32_t tw = op.tword[0], tb = op.tbit[0];
  double2 amp[ITEMS];
  // every load of the tile is issued before any is used
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    amp[it] = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < W; ++w) key[it][w] = 0;
    if (e < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) key[it][w] = in_keys.w[w][e];
      amp[it] = in_amp[e];
    }
  }
  // Group mode, NB = 1 or 2: when every entry of the tile has its partner at
  // e ^ 1, the partners are exchanged between lane pairs (e and e ^ 1 sit in
  // lanes t and t ^ 1 of one wave) and nothing is staged.  The partner found
  // is the one the staged search finds, so the results are the same.
  // Otherwise NB = 1 stages the tile (as NB = 0 always does) and NB = 2
  // returns false with nothing computed (s_stage is then never touched).
  bool aligned = false;
  double2 pamp[ITEMS];
  if (MODE == MODE_GROUP && NB != 0) {
    bool ok = true;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
      uint64_t pk[W];
#pragma unroll
      for (int w = 0; w < W; ++w) pk[w] = lane_pair_swap(key[it][w]);
      pamp[it].x = __longlong_as_double((long long)lane_pair_swap((uint64_t)__double_as_longlong(amp[it].x)));
      pamp[it].y = __longlong_as_double((long long)lane_pair_swap((uint64_t)__double_as_longlong(amp[it].y)));
      if (e < n) ok = ok && (e ^ 1ull) < n && same_idle<W>(key[it], pk, op.tmask);
    }
    aligned = __syncthreads_and(ok) != 0;
    if (NB == 2 && !aligned) return false;
  }
  if (MODE == MODE_GROUP && NB != 2 && !aligned) {
    // Neighbours come from LDS: slot 1 + i holds tile entry i, slot 0 the
    // entry before the tile and slot TILE + 1 the one after (when present).
    uint64_t* s_key = s_stage;
    double2* s_amp = reinterpret_cast<double2*>(s_stage + W * (TILE + 2));
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint32_t l = 1 + it * kBlock + threadIdx.x;
#pragma unroll
      for (int w = 0; w < W; ++w) s_key[w * (TILE + 2) + l] = key[it][w];
      s_amp[l] = amp[it];
    }
    if (threadIdx.x < 2) {
      const uint64_t e = threadIdx.x == 0 ? e0 - 1 : e0 + TILE;
      const uint32_t l = threadIdx.x == 0 ? 0 : TILE + 1;
      const bool ok = threadIdx.x == 0 ? e0 > 0 : e0 + TILE < n;
#pragma unroll
      for (int w = 0; w < W; ++w) s_key[w * (TILE + 2) + l] = ok ? in_keys.w[w][e] : 0ull;
      s_amp[l] = ok ? in_amp[e] : make_double2(0.0, 0.0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    keepm[it] = 0;
    out[it][0] = out[it][1] = make_double2(0.0, 0.0);
    if (e < n) {
      const double2 a = amp[it];
      const uint32_t b = (uint32_t)((sel_word<W>(key[it], tw) >> tb) & 1ull);
      // The matrix this entry's group gets: the op's own when its controls
      // hold, else the identity (the entry passes through); for a chain, the
      // product of the matrices of the ops whose controls hold, in op order.
      double mm[2][2];
      double mmi[2][2] = {{0.0, 0.0}, {0.0, 0.0}};   // imaginary parts (complex op only)
      if (op.nchain == 0) {
        const bool ctl = !op.has_ctl || controls_hold<W>(key[it], op.cmask, op.cval);
        mm[0][0] = ctl ? op.m[0][0] : 1.0;
        mm[0][1] = ctl ? op.m[0][1] : 0.0;
        mm[1][0] = ctl ? op.m[1][0] : 0.0;
        mm[1][1] = ctl ? op.m[1][1] : 1.0;
        if (op.cplx) {
          mmi[0][0] = ctl ? op.mi[0][0] : 0.0;
          mmi[0][1] = ctl ? op.mi[0][1] : 0.0;
          mmi[1][0] = ctl ? op.mi[1][0] : 0.0;
          mmi[1][1] = ctl ? op.mi[1][1] : 0.0;
        }
      } else {
        mm[0][0] = 1.0;
        mm[0][1] = 0.0;
        mm[1][0] = 0.0;
        mm[1][1] = 1.0;
        for (uint32_t q = 0; q < op.nchain; ++q) {
          const ChainStep& cs = op.chain[q];
          if (!controls_hold<W>(key[it], cs.cmask, cs.cval)) continue;
          const double t00 = cs.m[0][0] * mm[0][0] + cs.m[0][1] * mm[1][0];
          const double t01 = cs.m[0][0] * mm[0][1] + cs.m[0][1] * mm[1][1];
          const double t10 = cs.m[1][0] * mm[0][0] + cs.m[1][1] * mm[1][0];
          const double t11 = cs.m[1][0] * mm[0][1] + cs.m[1][1] * mm[1][1];
          mm[0][0] = t00;
          mm[0][1] = t01;
          mm[1][0] = t10;
          mm[1][1] = t11;
        }
      }
      {
        bool has_p = false;
        double2 ap = make_double2(0.0, 0.0);
        if (MODE == MODE_GROUP && aligned) {
          has_p = true;
          ap = pamp[it];
        } else if (MODE == MODE_GROUP && NB != 2) {
          // the partner is a neighbour on either side: grouped order keeps the
          // two members adjacent but not necessarily bit 0 first
          const uint64_t* s_key = s_stage;
          const double2* s_amp = reinterpret_cast<const double2*>(s_stage + W * (TILE + 2));
          const uint32_t l = 1 + it * kBlock + threadIdx.x;
          uint64_t pk[W], nk[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            pk[w] = s_key[w * (TILE + 2) + l - 1];
            nk[w] = s_key[w * (TILE + 2) + l + 1];
          }
          const bool prev_p = e > 0 && same_idle<W>(key[it], pk, op.tmask);
          const bool next_p = !prev_p && e + 1 < n && same_idle<W>(key[it], nk, op.tmask);
          has_p = prev_p || next_p;
          if (has_p) ap = s_amp[prev_p ? l - 1 : l + 1];
        }
        const double2 a0 = b == 0 ? a : ap;
        const double2 a1 = b == 0 ? ap : a;
#pragma unroll
        for (uint32_t r = 0; r < 2; ++r) {
          // a member of a full pair writes only the child with its own value
          if (has_p && r != b) continue;
          const double m0 = r ? mm[1][0] : mm[0][0];
          const double m1 = r ? mm[1][1] : mm[0][1];
          double2 v;
          bool nz0, nz1;
          if (op.cplx) {
            // complex matrix (a general rotation): same order, complex products
            const double i0 = r ? mmi[1][0] : mmi[0][0];
            const double i1 = r ? mmi[1][1] : mmi[0][1];
            const double2 p0 = cmul(a0, m0, i0), p1 = cmul(a1, m1, i1);
            v.x = p0.x + p1.x;
            v.y = p0.y + p1.y;
            nz0 = m0 != 0.0 || i0 != 0.0;
            nz1 = m1 != 0.0 || i1 != 0.0;
          } else {
            v.x = m0 * a0.x + m1 * a1.x;
            v.y = m0 * a0.y + m1 * a1.y;
            nz0 = m0 != 0.0;
            nz1 = m1 != 0.0;
          }
          const bool exists = has_p ? (nz0 || nz1) : (b ? nz1 : nz0);
          out[it][r] = v;
          if (exists && keep_amp(v.x, v.y, op.eps2)) keepm[it] |= 1u << r;
        }
      }
    }
  }
  return true;
}

// Write the kept children of one tile: the child of item `it` with target
// value r goes to pos[it] + (its rank among the item's kept children).
template <int W, int ITEMS>
__device__ __forceinline__ void pair_write(KeyPtrs<W>& out_keys, double2* __restrict__ out_amp, uint64_t cap,
                                           const GroupOp& op, const uint64_t (&key)[ITEMS][W],
                                           const double2 (&out)[ITEMS][2], const uint32_t (&keepm)[ITEMS],
                                           const uint64_t (&pos)[ITEMS], uint64_t (&orv)[W], uint64_t (&andv)[W]) {
  const uint32_t tw = op.tword[0];
  const uint64_t tbit = 1ull << op.tbit[0];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    uint64_t p = pos[it];
    if (keepm[it] == 3u && (p & 1ull) == 0 && p + 1 < cap) {
      // both children at an even position: one 16-byte store per key word
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t k0 = key[it][w], k1 = key[it][w];
        if ((uint32_t)w == tw) {
          k0 &= ~tbit;
          k1 |= tbit;
        }
        *reinterpret_cast<ulonglong2*>(&out_keys.w[w][p]) = make_ulonglong2(k0, k1);
        orv[w] |= k0 | k1;
        andv[w] &= k0 & k1;
      }
      out_amp[p] = out[it][0];
      out_amp[p + 1] = out[it][1];
      continue;
    }
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
      if (!((keepm[it] >> r) & 1u)) continue;
      uint64_t ok[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        ok[w] = key[it][w];
        if ((uint32_t)w == tw) ok[w] = r ? (ok[w] | tbit) : (ok[w] & ~tbit);
      }
      if (p < cap) {
#pragma unroll
        for (int w = 0; w < W; ++w) out_keys.w[w][p] = ok[w];
        out_amp[p] = out[it][r];
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        orv[w] |= ok[w];
        andv[w] &= ok[w];
      }
      ++p;
    }
  }
}

// The fused run of a one-target launch: the ops rops[0..rn) (generic records
// rgops) are applied to the kept children of every item before they are
// written at pos[it] (the upper child of an item that keeps both at pos + 1).
// Pass 0 takes the lower kept child of every item, pass 1 the upper child of
// items that keep both (in group mode: an entry without its partner whose
// matrix mixes); a wave runs pass 1 only when one of its lanes has such a
// child.  ONE: no item keeps both children (group mode with every partner in
// the neighbouring lane), so there is no pass 1.
template <int W, int ITEMS, bool ONE = false>
__device__ __forceinline__ void run_children(const GroupOp& op, const uint64_t (&key)[ITEMS][W],
                                             const double2 (&out)[ITEMS][2], const uint32_t (&keepm)[ITEMS],
                                             const uint64_t (&pos)[ITEMS], const FastOp* __restrict__ rops,
                                             uint32_t rn, const PermOp* __restrict__ rgops,
                                             KeyPtrs<W> out_keys, double2* __restrict__ out_amp, uint64_t cap,
                                             uint64_t (&orv)[W], uint64_t (&andv)[W]) {
  static_assert(W <= 2, "runs are fused for keys of at most 2 words");
  const uint32_t tw = op.tword[0];
  const uint64_t tbit = 1ull << op.tbit[0];
  // the children of one pass as 32-bit key halves and amplitudes
  auto load = [&](uint32_t pass, uint32_t (&h)[ITEMS][4], double2 (&ca)[ITEMS], bool (&has)[ITEMS]) {
    bool any = false;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint32_t km = keepm[it];
      has[it] = pass == 0 ? km != 0u : km == 3u;
      const uint32_t r = pass == 0 ? ((km & 1u) ? 0u : 1u) : 1u;
      h[it][2] = h[it][3] = 0u;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t v = key[it][w];
        if ((uint32_t)w == tw) v = r ? (v | tbit) : (v & ~tbit);
        h[it][2 * w] = (uint32_t)v;
        h[it][2 * w + 1] = (uint32_t)(v >> 32);
      }
      ca[it] = r ? out[it][1] : out[it][0];
      any = any || has[it];
    }
    return any;
  };
  uint32_t h0[ITEMS][4], h1[ITEMS][4];
  double2 a0[ITEMS], a1[ITEMS];
  bool has0[ITEMS], has1[ITEMS];
  (void)load(0, h0, a0, has0);
  run_ops<W, ITEMS, true>(h0, a0, rops, rn, rgops);
  const bool two = !ONE && __ballot(load(1, h1, a1, has1)) != 0ull;
  if (!ONE && two) run_ops<W, ITEMS, true>(h1, a1, rops, rn, rgops);
  // Both children of an item are written together: at an even position the
  // key words of the pair go out as one 16-byte store per word, so a wave's
  // stores cover whole lines instead of every other word.
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (!has0[it]) continue;
    const uint64_t p = pos[it];
    const bool pair = two && has1[it];
    uint64_t v0[W], v1[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      v0[w] = (uint64_t)h0[it][2 * w] | ((uint64_t)h0[it][2 * w + 1] << 32);
      v1[w] = (uint64_t)h1[it][2 * w] | ((uint64_t)h1[it][2 * w + 1] << 32);
      orv[w] |= v0[w];
      andv[w] &= v0[w];
      if (pair) {
        orv[w] |= v1[w];
        andv[w] &= v1[w];
      }
    }
    if (pair && (p & 1ull) == 0 && p + 1 < cap) {
#pragma unroll
      for (int w = 0; w < W; ++w)
        *reinterpret_cast<ulonglong2*>(&out_keys.w[w][p]) = make_ulonglong2(v0[w], v1[w]);
      out_amp[p] = a0[it];
      out_amp[p + 1] = a1[it];
    } else {
      if (p < cap) {
#pragma unroll
        for (int w = 0; w < W; ++w) out_keys.w[w][p] = v0[w];
        out_amp[p] = a0[it];
      }
      if (pair && p + 1 < cap) {
#pragma unroll
        for (int w = 0; w < W; ++w) out_keys.w[w][p + 1] = v1[w];
        out_amp[p + 1] = a1[it];
      }
    }
  }
}

// Speculative placement without look-back: when every entry of the op has
// exactly `f` kept children (f = 1: full pairs or pass-through in group mode;
// f = 2: both children in expand mode) the compacted position of entry e's
// children is f * e.  A tile that finds an entry with another count (or an
// output past the capacity) writes nothing and flags the launch; k_pair then
// compacts the whole op.  Tile = workgroup, no tickets.  RUN: the run that
// follows the op is applied to the children before they are written, as in
// the compacting launch (which, with RUN, then only counts its updates).
template <int W, int MODE, int ITEMS, bool RUN, int NB>
__global__ __launch_bounds__(kBlock, ITEMS >= 8 ? 4 : 1) void k_pair_spec(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                      KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                      uint32_t ns, uint64_t cap, GroupOp op, uint32_t f,
                                                      DevMeta* meta, uint32_t epoch, const FastOp* __restrict__ rops,
                                                      uint32_t rn, const PermOp* __restrict__ rgops) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  constexpr uint32_t kStageWords = MODE == MODE_GROUP && NB != 2 ? (W + 2) * (TILE + 2) : 1;
  __shared__ __align__(16) uint64_t s_stage[kStageWords];
  PrologueReads pr;
  if (launch_prologue_reads(meta, epoch, ns, false, &meta->spec_cool[MODE], &pr)) return;
  // cooling down after a wasted speculation: the compacting launch does the op
  if (pr.flag != 0u) {
    if (blockIdx.x == 0 && threadIdx.x == 0) meta->spec_irr[epoch % kRing] = kSpecSkipped;
    return;
  }
  const uint64_t n = pr.n;
  const uint64_t e0 = (uint64_t)blockIdx.x * TILE;
  if (e0 >= n) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (uint64_t)gridDim.x * TILE < n) raise_error(meta, kErrGrid, epoch);
  if (f * n > cap) {
    if (threadIdx.x == 0) meta->spec_irr[epoch % kRing] = 1u;
    return;
  }
  uint64_t key[ITEMS][W];
  double2 out[ITEMS][2];
  uint32_t keepm[ITEMS];
  if (!pair_tile<W, MODE, ITEMS, NB>(in_keys, in_amp, n, e0, op, s_stage, key, out, keepm)) {
    // partners not aligned (NB = 2): the compacting launch does the op
    if (threadIdx.x == 0) atomicOr(&meta->spec_irr[epoch % kRing], 1u);
    return;
  }
  bool reg = true;
  uint64_t pos[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    if (e < n && (uint32_t)__popc(keepm[it]) != f) reg = false;
    pos[it] = f * e;
  }
  if (!__syncthreads_and(reg)) {
    if (threadIdx.x == 0) atomicOr(&meta->spec_irr[epoch % kRing], 1u);
    return;
  }
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  // group mode with lane-pair partners (NB = 2): every entry keeps only its
  // own child
  if constexpr (RUN)
    run_children<W, ITEMS, MODE == MODE_GROUP && NB == 2>(op, key, out, keepm, pos, rops, rn, rgops, out_keys,
                                                           out_amp, cap, orv, andv);
  else
    pair_write<W, ITEMS>(out_keys, out_amp, cap, op, key, out, keepm, pos, orv, andv);
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// The compacting launch.  With spec_ep != 0 it follows k_pair_spec (launch
// spec_ep): when that launch met no irregular tile, its outputs stand and
// workgroup 0 only records the count f * n, the peak and the key masks.
// RUN: the run of non-branching ops that follows the op (rops[0..rn), generic
// records rgops) is applied to the kept children before they are written, in
// place of a separate permutation launch (keys of at most 2 words).  Children
// keep their positions, so the result equals the two launches bit for bit.
template <int W, int MODE, int ITEMS, bool RUN>
__global__ __launch_bounds__(kBlock) void k_pair(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                 KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                 uint32_t ns, uint64_t cap, GroupOp op, uint64_t* lb,
                                                 DevMeta* meta, uint32_t epoch, uint32_t xo, uint32_t spec_ep,
                                                 uint32_t f, const FastOp* __restrict__ rops, uint32_t rn,
                                                 const PermOp* __restrict__ rgops) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  // group mode: the tile's keys (W words) and amplitudes plus one entry on
  // each side, for the partner test; with RUN the same space then stages the
  // run's op records
  constexpr uint32_t kStageWords = MODE == MODE_GROUP ? (W + 2) * (TILE + 2) : 1;
  __shared__ __align__(16) uint64_t s_stage[kStageWords];
  uint64_t n;
  unsigned int sflag = 0u;
  if (!emit_begin(meta, ns, epoch, TILE, &n, xo, spec_ep != 0 ? &meta->spec_irr[spec_ep % kRing] : nullptr, &sflag))
    return;
  if (op.upd && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&meta->upd, (unsigned long long)(n * op.upd));
  if (sflag != 0u) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (sflag == kSpecSkipped) {
        const unsigned int c = meta->spec_cool[MODE];
        meta->spec_cool[MODE] = c ? c - 1u : 0u;
      } else {
        // the speculative launch was wasted: counted (the host stops trying at
        // its next read-back) and the next kSpecCool launches skip themselves
        atomicAdd(&meta->spec_fail[MODE], 1ull);
        meta->spec_cool[MODE] = kSpecCool;
      }
    }
  } else if (spec_ep != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const uint64_t m = f * n;
      meta->nnz_out[epoch % kRing] = m;
      meta->nring[(ns & 1) ^ 1] = m;
      atomicMax(&meta->peak, (unsigned long long)m);
      // (atomic: the op's own count above is added at the same time)
      if (RUN) atomicAdd(&meta->upd, (unsigned long long)(m * rn));
      for (int w = 0; w < kMaxW; ++w) {
        meta->or_mask[epoch % kRing][w] = meta->or_mask[spec_ep % kRing][w];
        meta->and_mask[epoch % kRing][w] = meta->and_mask[spec_ep % kRing][w];
      }
    }
    return;
  }
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;
  const uint64_t e0 = (uint64_t)tile * TILE;
  uint64_t key[ITEMS][W];
  double2 out[ITEMS][2];
  uint32_t keepm[ITEMS], cnt[ITEMS];
  pair_tile<W, MODE, ITEMS>(in_keys, in_amp, n, e0, op, s_stage, key, out, keepm);
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) cnt[it] = (uint32_t)__popc(keepm[it]);
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = ex + tile_total;
        if (ex + tile_total > cap) raise_error(meta, kErrCapacity, epoch);
        else atomicMax(&meta->peak, (unsigned long long)(ex + tile_total));
        // (atomic: workgroup 0 adds the op's own count at the same time)
        if (RUN) atomicAdd(&meta->upd, (unsigned long long)((ex + tile_total) * rn));
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  uint64_t pos[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) pos[it] = s_off + off[it];
  if constexpr (RUN) {
    // The tile's prefix is published (the look-back above), so later tiles do
    // not wait for this work.
    run_children<W, ITEMS>(op, key, out, keepm, pos, rops, rn, rgops, out_keys, out_amp, cap,
                                 orv, andv);
  } else {
    pair_write<W, ITEMS>(out_keys, out_amp, cap, op, key, out, keepm, pos, orv, andv);
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// k_filter: compaction with a keep predicate.
//   FILTER_PRUNE:   keep unless |a|^2 < eps^2 or a == 0
//   FILTER_COLLAPSE: entries of field value `fval` (on the given word/shift/mask)
//                    within instance `inst` are kept and divided by `scale`;
//                    other entries of that instance are dropped; entries of
//                    other instances pass unchanged.
//   FILTER_DROP_INST: drop every entry of instance `inst`.
// ---------------------------------------------------------------------------
enum { FILTER_PRUNE = 0, FILTER_COLLAPSE = 1, FILTER_DROP_INST = 2 };

struct FilterOp {
  uint32_t kind;
  uint32_t fword, fshift, iword, ishift, has_inst;
  uint32_t use_f, pad;
  uint64_t fmask, fval, imask, inst;
  double eps2, scale;
};

template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_filter(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                   KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                   uint32_t ns, uint64_t cap, FilterOp f, uint64_t* lb,
                                                   DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  uint64_t n;
  if (!emit_begin(meta, ns, epoch, TILE, &n, xo)) return;
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;
  uint64_t key[ITEMS][W];
  double2 a[ITEMS];
  uint32_t cnt[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = (uint64_t)tile * TILE + (uint64_t)it * kBlock + threadIdx.x;
    bool keep = false;
    a[it] = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < W; ++w) key[it][w] = 0;
    if (e < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) key[it][w] = in_keys.w[w][e];
      a[it] = in_amp[e];
      const bool mine = !f.has_inst || ((sel_word<W>(key[it], f.iword) >> f.ishift) & f.imask) == f.inst;
      if (f.kind == FILTER_PRUNE) {
        keep = !mine || keep_amp(a[it].x, a[it].y, f.eps2);
      } else if (f.kind == FILTER_COLLAPSE) {
        if (!mine) {
          keep = true;
        } else {
          keep = ((sel_word<W>(key[it], f.fword) >> f.fshift) & f.fmask) == f.fval;
          a[it].x = a[it].x / f.scale;
          a[it].y = a[it].y / f.scale;
        }
      } else {
        keep = !mine;
      }
    }
    cnt[it] = keep ? 1u : 0u;
  }
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = ex + tile_total;
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    if (!cnt[it]) continue;
    const uint64_t p = s_off + off[it];
    if (p < cap) {
#pragma unroll
      for (int w = 0; w < W; ++w) out_keys.w[w][p] = key[it][w];
      out_amp[p] = a[it];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      orv[w] |= key[it][w];
      andv[w] &= key[it][w];
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// Batched rounds: every instance follows its own op list.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ uint32_t inst_of(const uint64_t (&k)[W], uint32_t iword, uint32_t ishift, uint64_t imask) {
  return (uint32_t)((sel_word<W>(k, iword) >> ishift) & imask);
}

// Each entry runs its own instance's run of non-branching ops.  A wave takes
// the distinct instances among its lanes one at a time, so the op index stays
// uniform and the interpreter's dispatch stays scalar.  The grid is sized
// from the host's bound on the count, which after a round's reduction can be
// many times the count, so it is capped and strides over the entries.
template <int W, bool AMP>
__global__ __launch_bounds__(kBlock) void k_perm_batched(KeyPtrs<W> keys, double2* __restrict__ amp, uint32_t ns,
                                                         const FastOp* __restrict__ ops,
                                                         const PermOp* __restrict__ gops,
                                                         const RunRange* __restrict__ runs, uint32_t iword,
                                                         uint32_t ishift, uint64_t imask, uint32_t write_words,
                                                         DevMeta* meta, uint32_t epoch) {
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  if (launch_prologue(meta, epoch)) return;
  // the view [base, n) of the batched rounds
  const uint64_t vb = meta->base;
  const uint64_t n = meta->nring[ns & 1] - vb;
  offset_keys<W>(keys, vb);
  amp += vb;
  if ((uint64_t)blockIdx.x * kBlock >= n) return;
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0ull;
    andv[w] = ~0ull;
  }
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  // (the loop condition is uniform over the workgroup, which publishes its
  // masks once at the end)
  for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock; i0 < n; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    const bool valid = i < n;
    uint32_t h[1][4] = {{0u, 0u, 0u, 0u}};
    double2 a[1] = {make_double2(0.0, 0.0)};
    uint64_t k[W];
#pragma unroll
    for (int w = 0; w < W; ++w) k[w] = valid ? keys.w[w][i] : 0ull;
    const uint32_t inst = valid ? inst_of<W>(k, iword, ishift, imask) : 0u;
    const RunRange rr = valid ? runs[inst] : RunRange{0u, 0u};
    if (W <= 2) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        h[0][2 * w] = (uint32_t)k[w];
        h[0][2 * w + 1] = (uint32_t)(k[w] >> 32);
      }
    }
    if (AMP && valid) a[0] = amp[i];
    uint64_t pending = __ballot(valid && rr.len > 0);
    while (pending) {
      const uint32_t lead = (uint32_t)__builtin_ctzll(pending);
      const uint32_t u = __builtin_amdgcn_readfirstlane(__shfl(inst, (int)lead, 64));
      const bool mine = valid && rr.len > 0 && inst == u;
      pending &= ~__ballot(mine);
      if (mine) {
        const uint32_t start = __builtin_amdgcn_readfirstlane(rr.start);
        const uint32_t len = __builtin_amdgcn_readfirstlane(rr.len);
        for (uint32_t o = start; o < start + len; ++o) {
          const FastOp rec = load_rec(ops + o);
          if (W <= 2) fast_step<W, 1, AMP>(h, a, rec, gops);
          else perm_apply<W>(k, a[0], gops[rec.e]);
        }
      }
    }
    if (W <= 2) {
#pragma unroll
      for (int w = 0; w < W; ++w) k[w] = (uint64_t)h[0][2 * w] | ((uint64_t)h[0][2 * w + 1] << 32);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (valid) {
        orv[w] |= k[w];
        andv[w] &= k[w];
      }
      if (valid && (write_words & (1u << w))) keys.w[w][i] = k[w];
    }
    if (AMP && valid) amp[i] = a[0];
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// The op record of an instance in a batched round, read through pointer type
// P: a constant address space pointer when every entry of the wave's row
// belongs to one instance (each field one scalar load, held in scalar
// registers), else a plain global pointer (per-lane loads).
typedef const __attribute__((address_space(4))) BatchOp ConstBatchOp;

// Children of one parent: the target bits' current values (bits) and the
// number of children reached through nonzero elements (product over the
// targets of the nonzero entries in column b_j); a parent whose controls fail,
// or whose instance has no branching op this round, is copied (copy, 1 child).
template <int W, class P>
__device__ __forceinline__ uint32_t expand_count(P op, const uint64_t (&key)[W], uint32_t& bits, bool& copy) {
  const uint32_t k = op->k;
  bool ctl = true;
  if (op->has_ctl) {
#pragma unroll
    for (int w = 0; w < W; ++w) ctl = ctl && ((key[w] & op->cmask[w]) == op->cval[w]);
  }
  copy = k == 0 || !ctl;
  bits = 0;
  if (copy) return 1u;
  const bool cplx = op->cplx != 0u;
  uint32_t cnt = 1;
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t bj = (uint32_t)((sel_word<W>(key, op->tword[j]) >> op->tbit[j]) & 1ull);
    bits |= bj << j;
    const bool c0 = (bj ? op->m[0][1] : op->m[0][0]) != 0.0 || (cplx && (bj ? op->mi[0][1] : op->mi[0][0]) != 0.0);
    const bool c1 = (bj ? op->m[1][1] : op->m[1][0]) != 0.0 || (cplx && (bj ? op->mi[1][1] : op->mi[1][0]) != 0.0);
    cnt *= (uint32_t)c0 + (uint32_t)c1;
  }
  return cnt;
}

// Child r of one parent (the r-th of its existing children in ascending order
// of the target bits' new values s, lowest target least significant): a
// target whose column has two nonzero elements takes the next bit of r, one
// with a single nonzero element its row; the amplitude is multiplied by the
// elements stage by stage in ascending target order.  A copied parent is its
// own only child.
template <int W, class P>
__device__ __forceinline__ void expand_child(P op, const uint64_t (&key)[W], double2 a, uint32_t bits, bool copy,
                                             uint32_t r, uint64_t (&ok)[W], double2& v) {
#pragma unroll
  for (int w = 0; w < W; ++w) ok[w] = key[w];
  v = a;
  if (copy) return;
  const uint32_t k = op->k;
  const bool cplx = op->cplx != 0u;
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t bj = (bits >> j) & 1u;
    const double c0 = bj ? op->m[0][1] : op->m[0][0];
    const double c1 = bj ? op->m[1][1] : op->m[1][0];
    const double i0 = cplx ? (bj ? op->mi[0][1] : op->mi[0][0]) : 0.0;
    const double i1 = cplx ? (bj ? op->mi[1][1] : op->mi[1][0]) : 0.0;
    const bool nz0 = c0 != 0.0 || i0 != 0.0;
    const bool nz1 = c1 != 0.0 || i1 != 0.0;
    uint32_t sj;
    if (nz0 && nz1) {
      sj = r & 1u;
      r >>= 1;
    } else {
      sj = nz1 ? 1u : 0u;
    }
    const double c = sj ? c1 : c0;
    if (cplx) {
      v = cmul(v, c, sj ? i1 : i0);
    } else {
      v.x = c * v.x;
      v.y = c * v.y;
    }
    const uint64_t bit = 1ull << op->tbit[j];
    const uint32_t tw = op->tword[j];
#pragma unroll
    for (int w = 0; w < W; ++w)
      if ((uint32_t)w == tw) ok[w] = sj ? (ok[w] | bit) : (ok[w] & ~bit);
  }
}

__device__ __forceinline__ uint32_t lane_read(uint32_t lane, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(lane << 2), (int)v);
}
__device__ __forceinline__ uint64_t lane_read64(uint32_t lane, uint64_t v) {
  return (uint64_t)lane_read(lane, (uint32_t)v) | ((uint64_t)lane_read(lane, (uint32_t)(v >> 32)) << 32);
}

// Branch expansion: every parent emits the children of its instance's op
// (expand_count / expand_child).  Output offsets come from a look-back prefix
// of the per-parent child counts.  ITEMS parents per thread, all loads of the
// tile issued before any is used.  Entries are ordered by instance, so almost
// every row of 64 entries belongs to one instance, whose record the row then
// reads with scalar loads.
template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_expand_batched(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                           KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                           uint32_t ns, uint64_t cap, const BatchOp* __restrict__ bops,
                                                           uint32_t iword, uint32_t ishift, uint64_t imask,
                                                           uint64_t* lb, DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  uint64_t n, vb;
  if (!emit_begin_view(meta, ns, epoch, TILE, &n, &vb, xo)) return;
  offset_keys<W>(in_keys, vb);
  offset_keys<W>(out_keys, vb);
  in_amp += vb;
  out_amp += vb;
  cap -= vb;
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;
  const uint64_t e0 = (uint64_t)tile * TILE;
  ConstBatchOp* const cbops = (ConstBatchOp*)bops;
  uint64_t key[ITEMS][W];
  double2 a[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    a[it] = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < W; ++w) key[it][w] = 0;
    if (e < n) {
#pragma unroll
      for (int w = 0; w < W; ++w) key[it][w] = in_keys.w[w][e];
      a[it] = in_amp[e];
    }
  }
  uint32_t bits[ITEMS], cnt[ITEMS], inst[ITEMS];
  bool copy[ITEMS];
  uint32_t uni = 0;   // bit it: the row of item it holds one instance
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    inst[it] = e < n ? inst_of<W>(key[it], iword, ishift, imask) : 0u;
    const uint32_t u = __builtin_amdgcn_readfirstlane(inst[it]);
    const bool one = __ballot(e < n && inst[it] != u) == 0ull;
    uni |= (one ? 1u : 0u) << it;
    bits[it] = 0;
    cnt[it] = 0;
    copy[it] = true;
    if (e < n) {
      if (one) cnt[it] = expand_count<W>(cbops + u, key[it], bits[it], copy[it]);
      else cnt[it] = expand_count<W>(bops + inst[it], key[it], bits[it], copy[it]);
    }
  }
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = vb + ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = vb + ex + tile_total;
        if (ex + tile_total > cap) raise_error(meta, kErrCapacity, epoch);
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  // The children of one row of 64 parents fill a contiguous output range,
  // which the row writes 64 slots at a time, lane l slot t = base + l: its
  // parent is the last lane whose first child is at or before t (a binary
  // search over the row's offsets, read across lanes with ds_bpermute), its
  // child the (t - that offset)-th; consecutive lanes write consecutive
  // outputs.  Every lane of the wave takes part in each step.
  const uint32_t lane = lane_id();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint32_t rb = __builtin_amdgcn_readfirstlane(off[it]);
    const uint32_t rt = (uint32_t)__builtin_amdgcn_readlane((int)(off[it] + cnt[it]), 63) - rb;
    const uint32_t x = off[it] - rb;
    const uint32_t cf = copy[it] ? 1u : 0u;
    const uint64_t p0 = s_off + rb;
    const bool one = (uni >> it) & 1u;
    const uint32_t u = __builtin_amdgcn_readfirstlane(inst[it]);
    for (uint32_t base = 0; base < rt; base += 64) {
      const uint32_t t = base + lane;
      uint32_t j = 0;
#pragma unroll
      for (uint32_t step = 32; step; step >>= 1)
        if (lane_read(j + step, x) <= t) j += step;
      const uint32_t xj = lane_read(j, x);
      uint64_t pk[W];
#pragma unroll
      for (int w = 0; w < W; ++w) pk[w] = lane_read64(j, key[it][w]);
      double2 pa;
      pa.x = __longlong_as_double((long long)lane_read64(j, (uint64_t)__double_as_longlong(a[it].x)));
      pa.y = __longlong_as_double((long long)lane_read64(j, (uint64_t)__double_as_longlong(a[it].y)));
      const uint32_t pb = lane_read(j, bits[it]);
      const bool pc = lane_read(j, cf) != 0u;
      const uint32_t pi = lane_read(j, inst[it]);
      if (t < rt) {
        uint64_t ok[W];
        double2 v;
        if (one) expand_child<W>(cbops + u, pk, pa, pb, pc, t - xj, ok, v);
        else expand_child<W>(bops + pi, pk, pa, pb, pc, t - xj, ok, v);
        const uint64_t q = p0 + t;
        if (q < cap) {
#pragma unroll
          for (int w = 0; w < W; ++w) out_keys.w[w][q] = ok[w];
          out_amp[q] = v;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          orv[w] |= ok[w];
          andv[w] &= ok[w];
        }
      }
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// Reduce-by-key over sorted candidates: the first entry of each run of equal
// keys sums the run left to right; instances that branched this round drop
// sums with |a|^2 < eps^2 or a == 0.  One output per run, compacted.  A run
// has at most 2^5 members (one branching op of up to five targets per
// instance and round), so the tile is staged in LDS with the entry before it
// and the kRunHalo entries after it.  Runs are long after a many-target
// expansion (most entries are not heads), so the heads are first compacted
// in entry order and thread t sums the runs of heads t, t + kBlock, ...: the
// summing loops run on busy lanes, and the kept sums go out consecutively.
constexpr uint32_t kRunHalo = 64;

template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_reduce_batched(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                           KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                           uint32_t ns, uint64_t cap, const BatchOp* __restrict__ bops,
                                                           uint32_t iword, uint32_t ishift, uint64_t imask,
                                                           uint64_t* lb, DevMeta* meta, uint32_t epoch, uint32_t xo) {
  constexpr uint32_t TILE = kBlock * ITEMS;
  constexpr uint32_t S = TILE + 1 + kRunHalo;   // staged slots: [e0 - 1, e0 + TILE + kRunHalo)
  static_assert(S < 65536, "slot indices are 16-bit");
  __shared__ uint32_t s_wtot[ITEMS][kBlock / 64];
  __shared__ uint64_t s_off;
  __shared__ uint64_t s_lb[12];
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_key[W * S];
  __shared__ double2 s_amp[S];
  __shared__ uint16_t s_head[TILE];   // slot of the tile's h-th run head
  uint64_t n, vb;
  if (!emit_begin_view(meta, ns, epoch, TILE, &n, &vb, xo)) return;
  offset_keys<W>(in_keys, vb);
  offset_keys<W>(out_keys, vb);
  in_amp += vb;
  out_amp += vb;
  cap -= vb;
  const uint32_t tile = take_tile(meta, epoch, &s_tile, xo);
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  if (tile_out_of_range(tile, ntiles, &meta->err, xo)) return;
  const uint64_t e0 = (uint64_t)tile * TILE;
  // stage slot l = entry e0 - 1 + l (zero key, zero amplitude past n); all
  // loads first, then the LDS stores
  constexpr uint32_t R = (S + kBlock - 1) / kBlock;
  uint64_t sk[R][W];
  double2 sa[R];
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t l = r * kBlock + threadIdx.x;
    const uint64_t e = e0 + l - 1;
    const bool ok = l < S && (l > 0 || e0 > 0) && e < n;
#pragma unroll
    for (int w = 0; w < W; ++w) sk[r][w] = ok ? in_keys.w[w][e] : 0ull;
    sa[r] = ok ? in_amp[e] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t l = r * kBlock + threadIdx.x;
    if (l < S) {
#pragma unroll
      for (int w = 0; w < W; ++w) s_key[w * S + l] = sk[r][w];
      s_amp[l] = sa[r];
    }
  }
  __syncthreads();
  // run heads of the tile's entries, numbered in entry order
  uint32_t hf[ITEMS], hoff[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint32_t l = 1 + it * kBlock + threadIdx.x;
    const uint64_t e = e0 + l - 1;
    hf[it] = 0;
    if (e < n) {
      bool eq = e > 0;
#pragma unroll
      for (int w = 0; w < W; ++w) eq = eq && s_key[w * S + l - 1] == s_key[w * S + l];
      hf[it] = eq ? 0u : 1u;
    }
  }
  const uint32_t nh = (uint32_t)tile_offsets<ITEMS>(hf, hoff, s_wtot);
#pragma unroll
  for (int it = 0; it < ITEMS; ++it)
    if (hf[it]) s_head[hoff[it]] = (uint16_t)(1 + it * kBlock + threadIdx.x);
  __syncthreads();
  // thread t: heads t + j * kBlock
  ConstBatchOp* const cbops = (ConstBatchOp*)bops;
  uint64_t key[ITEMS][W];
  double2 sum[ITEMS];
  uint32_t cnt[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t h = j * kBlock + threadIdx.x;
    const bool act = h < nh;
    const uint32_t l = act ? s_head[h] : 1u;
    const uint64_t e = e0 + l - 1;
#pragma unroll
    for (int w = 0; w < W; ++w) key[j][w] = act ? s_key[w * S + l] : 0ull;
    sum[j] = make_double2(0.0, 0.0);
    cnt[j] = 0;
    // the wave's one instance (scalar loads of its record), if it has one
    const uint32_t inst = inst_of<W>(key[j], iword, ishift, imask);
    const uint32_t u = __builtin_amdgcn_readfirstlane(inst);
    const bool one = __ballot(act && inst != u) == 0ull;
    if (act) {
      double2 acc = s_amp[l];
      for (uint32_t m = 1; m <= kRunHalo - 1 && e + m < n; ++m) {
        bool eq = true;
#pragma unroll
        for (int w = 0; w < W; ++w) eq = eq && s_key[w * S + l + m] == key[j][w];
        if (!eq) break;
        const double2 x = s_amp[l + m];
        acc.x = acc.x + x.x;
        acc.y = acc.y + x.y;
      }
      sum[j] = acc;
      const bool prune = one ? cbops[u].prune != 0u : bops[inst].prune != 0u;
      const double eps2 = one ? cbops[u].eps2 : bops[inst].eps2;
      cnt[j] = (prune ? keep_amp(acc.x, acc.y, eps2) : true) ? 1u : 0u;
    }
  }
  // kept sums in head order (= entry order)
  uint32_t off[ITEMS];
  const uint64_t tile_total = tile_offsets<ITEMS>(cnt, off, s_wtot);
  {
    const uint64_t ex = lookback_block(lb, tile, tile_total, epoch, &meta->err, s_lb);
    if (threadIdx.x == 0) {
      s_off = ex;
      if (tile == ntiles - 1) {
        meta->nnz_out[epoch % kRing] = vb + ex + tile_total;
        meta->nring[(ns & 1) ^ 1] = vb + ex + tile_total;
        atomicMax(&meta->peak, (unsigned long long)(vb + ex + tile_total));
      }
    }
  }
  __syncthreads();
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (!cnt[j]) continue;
    const uint64_t p = s_off + off[j];
    if (p < cap) {
#pragma unroll
      for (int w = 0; w < W; ++w) out_keys.w[w][p] = key[j][w];
      out_amp[p] = sum[j];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      orv[w] |= key[j][w];
      andv[w] &= key[j][w];
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// ---------------------------------------------------------------------------
// Retiring finished instances (batched rounds).  Instances are relabelled so
// that labels ascend with the round in which an instance runs its last op;
// the entries are sorted by (label, key) after every round, so the finished
// instances form a prefix that later rounds leave alone.
// ---------------------------------------------------------------------------

// Instance field := map[instance field] on every entry [0, n) (in place; the
// view base is ignored).  With `reset_base` the retired prefix is given back
// to the whole array (base = 0) and generation `gen` records that.
template <int W>
__global__ __launch_bounds__(kBlock) void k_relabel(KeyPtrs<W> keys, uint32_t ns, uint32_t iword, uint32_t ishift,
                                                    uint64_t imask, const uint32_t* __restrict__ map,
                                                    uint32_t reset_base, uint32_t gen, DevMeta* meta,
                                                    uint32_t epoch) {
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  if (launch_prologue(meta, epoch)) return;
  const uint64_t n = meta->nring[ns & 1];
  if (reset_base && blockIdx.x == 0 && threadIdx.x == 0) {
    meta->base = 0;
    meta->base_gen[gen % kBaseGens] = 0;
  }
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    uint64_t k[W];
#pragma unroll
    for (int w = 0; w < W; ++w) k[w] = keys.w[w][i];
    const uint32_t l = map[inst_of<W>(k, iword, ishift, imask)];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if ((uint32_t)w == iword) {
        k[w] = (k[w] & ~(imask << ishift)) | ((uint64_t)l << ishift);
        keys.w[w][i] = k[w];
      }
      orv[w] |= k[w];
      andv[w] &= k[w];
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

// Retire the labels below `a`: find p, the first entry of [base, n) whose
// label is at least `a` (entries are sorted by label), and copy [base, p)
// from the current buffer to the other one, so both hold the final prefix.
// Every workgroup finds p itself (one wave, a 64-way search over the sorted
// labels); workgroup 0 leaves it in retire_p for k_retire_set.
template <int W>
__global__ __launch_bounds__(kBlock) void k_retire_copy(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                        KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                        uint32_t ns, uint32_t iword, uint32_t ishift, uint64_t imask,
                                                        uint32_t a, DevMeta* meta, uint32_t epoch) {
  __shared__ uint64_t s_p;
  if (launch_prologue(meta, epoch)) return;
  const uint64_t base = meta->base;
  const uint64_t n = meta->nring[ns & 1];
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    const uint64_t* lw = in_keys.w[iword];
    // invariant: the first entry with label >= a lies in [lo, hi] (hi = n: none)
    uint64_t lo = base, hi = n;
    while (hi > lo) {
      const uint64_t len = hi - lo;
      const uint64_t step = (len + 63) / 64;
      const uint64_t q = lo + (uint64_t)(lane + 1) * step - 1;
      const bool probe = q < hi;
      const bool ge = probe && (uint32_t)((lw[q] >> ishift) & imask) >= a;
      // labels ascend, so the probes below the first ">= a" are a prefix of the lanes
      const uint64_t below = __ballot(probe && !ge);
      const uint32_t f = (uint32_t)__popcll(below);
      const uint64_t nlo = f == 0 ? lo : lo + (uint64_t)f * step;
      const uint64_t qf = lo + (uint64_t)(f + 1) * step - 1;
      const uint64_t nhi = (f < 64 && qf < hi) ? qf : hi;
      if (step == 1) {
        lo = nlo;
        hi = nlo;
      } else {
        lo = nlo;
        hi = nhi;
      }
    }
    if (lane == 0) s_p = lo;
  }
  __syncthreads();
  const uint64_t p = s_p;
  if (blockIdx.x == 0 && threadIdx.x == 0) meta->retire_p = p;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = base + (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < p; i += stride) {
#pragma unroll
    for (int w = 0; w < W; ++w) out_keys.w[w][i] = in_keys.w[w][i];
    out_amp[i] = in_amp[i];
  }
}

// base = retire_p (one thread, after every workgroup of k_retire_copy has
// read the old base), or 0 with `zero` (the rounds are over); generation
// `gen` records it for the host's accounting.
static __global__ void k_retire_set(DevMeta* meta, uint32_t gen, uint32_t zero) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*reinterpret_cast<volatile unsigned int*>(&meta->err) != 0u) return;
  const unsigned long long b = zero ? 0ull : meta->retire_p;
  meta->base = b;
  meta->base_gen[gen % kBaseGens] = b;
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
static __global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static __global__ void k_ring_init(DevMeta* meta) {
  if (blockIdx.x != 0) return;
  for (int r = threadIdx.x; r < kRing; r += blockDim.x) {
    meta->counters[r] = 0;
    meta->spec_irr[r] = 0;
    for (int x = 0; x < kXcds; ++x) meta->xcd_ctr[r][x * kXcdStride] = 0;
    meta->nnz_out[r] = 0;
    for (int w = 0; w < kMaxW; ++w) {
      meta->or_mask[r][w] = 0;
      meta->and_mask[r][w] = ~0ull;
    }
  }
}

// Check point of a replayed graph: the entry count in slot `ns` must equal the
// count the plan was made for, and (mask_slot >= 0) the key bits that vary
// over the entries, per the OR / AND masks in that ring slot, must lie inside
// `allowed`.  Otherwise raise kErrPlan tagged `epoch`; every later launch then
// changes nothing.  An earlier error takes precedence.
static __global__ void k_plan_guard(DevMeta* meta, uint32_t ns, uint64_t n_expect, int mask_slot, PlanVar allowed,
                             uint32_t epoch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*reinterpret_cast<volatile unsigned int*>(&meta->err) != 0u) return;
  bool bad = meta->nring[ns & 1] != n_expect;
  if (mask_slot >= 0)
    for (int w = 0; w < kMaxW; ++w)
      bad = bad || ((meta->or_mask[mask_slot][w] & ~meta->and_mask[mask_slot][w]) & ~allowed.var[w]) != 0ull;
  if (bad) raise_error(meta, kErrPlan, epoch);
}

// Copy the entries of slot `ns` (count read on the device) to the other
// buffer and count slot.  Does nothing after an error.
template <int W>
__global__ __launch_bounds__(kBlock) void k_copy_state(KeyPtrs<W> in_keys, const double2* __restrict__ in_amp,
                                                       KeyPtrs<W> out_keys, double2* __restrict__ out_amp,
                                                       uint32_t ns, DevMeta* meta) {
  if (*reinterpret_cast<volatile unsigned int*>(&meta->err) != 0u) return;
  const uint64_t n = meta->nring[ns & 1];
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int w = 0; w < W; ++w) out_keys.w[w][i] = in_keys.w[w][i];
    out_amp[i] = in_amp[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) meta->nring[(ns & 1) ^ 1] = n;
}

// XCD of each of the first gridDim.x workgroups (checks the round-robin spread).
static __global__ void k_xcc_probe(uint64_t* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

static __global__ void k_clear_err(DevMeta* meta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    meta->err = 0;
    meta->err_epoch = 0;
  }
}

// Host-known entry count into ring slot `ns` (after imports and rebinds).
static __global__ void k_set_n(DevMeta* meta, uint32_t ns, uint64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    meta->nring[ns & 1] = n;
    if (n > meta->peak) meta->peak = n;
  }
}

// OR / AND of all keys, for when the masks of the launch that produced the
// entries have left the ring.
template <int W>
__global__ __launch_bounds__(kBlock) void k_masks(KeyPtrs<W> keys, uint32_t ns, uint64_t cap, DevMeta* meta,
                                                  uint32_t epoch) {
  __shared__ uint64_t s_red[2 * kMaxW * 4];
  if (launch_prologue(meta, epoch)) return;
  const uint64_t nr = meta->nring[ns & 1];
  const uint64_t n = nr < cap ? nr : cap;
  uint64_t orv[W], andv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    orv[w] = 0;
    andv[w] = ~0ull;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint64_t v = keys.w[w][i];
      orv[w] |= v;
      andv[w] &= v;
    }
  }
  publish_masks<W>(meta, epoch, orv, andv, s_red);
}

static __global__ void k_meta_init(DevMeta* meta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int r = 0; r < kRing; ++r) {
      meta->counters[r] = 0;
      meta->spec_irr[r] = 0;
      for (int x = 0; x < kXcds; ++x) meta->xcd_ctr[r][x * kXcdStride] = 0;
      meta->nnz_out[r] = 0;
      for (int w = 0; w < kMaxW; ++w) {
        meta->or_mask[r][w] = 0;
        meta->and_mask[r][w] = ~0ull;
      }
    }
    meta->peak = 0;
    meta->upd = 0;
    meta->base = 0;
    meta->retire_p = 0;
    for (int g = 0; g < kBaseGens; ++g) meta->base_gen[g] = 0;
    meta->spec_fail[0] = meta->spec_fail[1] = 0;
    meta->spec_cool[0] = meta->spec_cool[1] = 0;
    meta->nring[0] = meta->nring[1] = 0;
    meta->err = 0;
    meta->err_epoch = 0;
  }
}

// Pack register values (n x nregs, row-major) into keys and append them at
// position `at`; the instance field gets `inst` (has_inst == 1) or `inst`
// plus the row index (has_inst == 2).
struct PackDesc {
  uint32_t nregs, has_inst, iword, ishift;
  uint64_t inst;
  uint32_t word[64], shift[64];
  uint64_t mask[64];
};

template <int W>
__global__ void k_pack(const uint64_t* __restrict__ values, const double2* __restrict__ amps, uint64_t n,
                       KeyPtrs<W> keys, double2* __restrict__ amp, uint64_t at, PackDesc pd) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k[W];
#pragma unroll
  for (int w = 0; w < W; ++w) k[w] = 0;
  for (uint32_t r = 0; r < pd.nregs; ++r) {
    const uint64_t v = values[i * pd.nregs + r] & pd.mask[r];
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (pd.word[r] == (uint32_t)w) k[w] |= v << pd.shift[r];
  }
  if (pd.has_inst) {
    const uint64_t iv = pd.has_inst == 2 ? pd.inst + i : pd.inst;
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (pd.iword == (uint32_t)w) k[w] |= iv << pd.ishift;
  }
#pragma unroll
  for (int w = 0; w < W; ++w) keys.w[w][at + i] = k[w];
  amp[at + i] = amps[i];
}

// Copy entries [lo, hi) of instance-sorted keys into a W-interleaved export
// buffer with the instance field cleared.
template <int W>
__global__ void k_export(KeyPtrs<W> keys, const double2* __restrict__ amp, uint64_t lo, uint64_t hi,
                         uint64_t* __restrict__ out_keys, double2* __restrict__ out_amp,
                         uint32_t iword, uint64_t iclear) {
  const uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= hi) return;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t v = keys.w[w][i];
    if ((uint32_t)w == iword) v &= ~iclear;
    out_keys[(i - lo) * W + w] = v;
  }
  out_amp[i - lo] = amp[i];
}

// Per-instance entry ranges of an instance-sorted state: bounds[inst] = first
// index with instance >= inst (bounds has ninst + 1 slots, pre-filled with n).
template <int W>
__global__ void k_inst_bounds(KeyPtrs<W> keys, uint64_t n, uint32_t iword, uint32_t ishift,
                              uint64_t imask, uint64_t* bounds, uint32_t ninst) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k[W];
#pragma unroll
  for (int w = 0; w < W; ++w) k[w] = keys.w[w][i];
  const uint64_t cur = (sel_word<W>(k, iword) >> ishift) & imask;
  uint64_t prv = 0;
  if (i > 0) {
    uint64_t pk[W];
#pragma unroll
    for (int w = 0; w < W; ++w) pk[w] = keys.w[w][i - 1];
    prv = (sel_word<W>(pk, iword) >> ishift) & imask;
  } else {
    prv = 0;
    for (uint64_t j = 0; j <= cur && j < ninst; ++j) bounds[j] = 0;
    return;
  }
  // instances prv+1 .. cur start here
  for (uint64_t j = prv + 1; j <= cur && j < ninst; ++j) bounds[j] = i;
}

// ---------------------------------------------------------------------------
// measurement support (a register field of one instance)
// ---------------------------------------------------------------------------
// Tile sums of w_i = |a_i|^2 over the entries of the instance (0 elsewhere),
// in a fixed order per tile.
template <int W>
__global__ __launch_bounds__(kBlock) void k_prob_tiles(KeyPtrs<W> keys, const double2* __restrict__ amp,
                                                       uint64_t n, FilterOp f, double* __restrict__ tile_sum) {
  __shared__ double s_scan[4];
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  double w = 0.0;
  if (e < n) {
    uint64_t k[W];
#pragma unroll
    for (int j = 0; j < W; ++j) k[j] = keys.w[j][e];
    const bool mine = !f.has_inst || ((sel_word<W>(k, f.iword) >> f.ishift) & f.imask) == f.inst;
    const bool pick = !f.use_f || ((sel_word<W>(k, f.fword) >> f.fshift) & f.fmask) == f.fval;
    const double2 a = amp[e];
    if (mine && pick) w = a.x * a.x + a.y * a.y;
  }
  double tot;
  block_excl_scan<double>(w, s_scan, tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Sequential exclusive scan of the tile sums (one thread; fixed order).
static __global__ void k_prob_scan(double* tile_sum, uint64_t ntiles, double* total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double run = 0.0;
  for (uint64_t t = 0; t < ntiles; ++t) {
    const double x = tile_sum[t];
    tile_sum[t] = run;
    run = run + x;
  }
  *total = run;
}

// Each entry of the instance gets its inclusive running sum (ascending field
// order).  The outcome is the field value of the first entry (lowest index)
// whose running sum exceeds u*P: out[0] gets that index by an atomic minimum,
// so exactly one entry is chosen even where rounding makes the sums of
// neighbouring entries overlap or leave a gap.  out[2] gets the largest field
// value with weight, the outcome when no running sum exceeds u*P (u*P at the
// total by rounding).
template <int W>
__global__ __launch_bounds__(kBlock) void k_prob_find(KeyPtrs<W> keys, const double2* __restrict__ amp,
                                                      uint64_t n, FilterOp f, const double* __restrict__ tile_pre,
                                                      const double* __restrict__ total, double u,
                                                      double* __restrict__ incl, unsigned long long* out) {
  __shared__ double s_scan[4];
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  double w = 0.0;
  bool mine = false;
  uint64_t fv = 0;
  if (e < n) {
    uint64_t k[W];
#pragma unroll
    for (int j = 0; j < W; ++j) k[j] = keys.w[j][e];
    mine = !f.has_inst || ((sel_word<W>(k, f.iword) >> f.ishift) & f.imask) == f.inst;
    fv = (sel_word<W>(k, f.fword) >> f.fshift) & f.fmask;
    const double2 a = amp[e];
    if (mine) w = a.x * a.x + a.y * a.y;
  }
  double tot;
  const double ex = block_excl_scan<double>(w, s_scan, tot);
  if (e < n) {
    const double after = (tile_pre[blockIdx.x] + ex) + w;
    incl[e] = after;
    const double target = u * (*total);
    if (mine && w > 0.0) {
      atomicMax(&out[2], (unsigned long long)fv);
      if (after > target) atomicMin(&out[0], (unsigned long long)e);
    }
  }
}

// Field value of the chosen entry (out[0]) into out[1].
template <int W>
__global__ void k_prob_pick(KeyPtrs<W> keys, FilterOp f, unsigned long long* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t e = out[0];
  if (e == ~0ull) return;
  uint64_t k[W];
#pragma unroll
  for (int j = 0; j < W; ++j) k[j] = keys.w[j][e];
  out[1] = (sel_word<W>(k, f.fword) >> f.fshift) & f.fmask;
}

// ---------------------------------------------------------------------------
// Probability readout without collapse (entries sorted by instance and the
// register's field): per-field sums of |a|^2 in a fixed order.
// ---------------------------------------------------------------------------
// Segmented inclusive sums inside each tile of kBlock entries: a segment
// starts where (instance, field) changes.  part[e] = sum from the segment's
// start (or the tile's) to e; fhead[t] = position of the tile's first segment
// start (kBlock if none); tail[t] = part of the tile's last entry.
template <int W>
__global__ __launch_bounds__(kBlock) void k_runs_tile(KeyPtrs<W> keys, const double2* __restrict__ amp, uint64_t n,
                                                      FilterOp f, double* __restrict__ part,
                                                      uint32_t* __restrict__ fhead, double* __restrict__ tail) {
  __shared__ double s_v[kBlock / 64];
  __shared__ uint32_t s_f[kBlock / 64];
  __shared__ uint32_t s_head;
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_head = kBlock;
  double v = 0.0;
  uint32_t head = 0;
  if (e < n) {
    uint64_t k[W];
#pragma unroll
    for (int j = 0; j < W; ++j) k[j] = keys.w[j][e];
    const uint64_t ii = f.has_inst ? ((sel_word<W>(k, f.iword) >> f.ishift) & f.imask) : 0;
    const uint64_t fv = (sel_word<W>(k, f.fword) >> f.fshift) & f.fmask;
    if (!f.has_inst || ii == f.inst) {
      const double2 a = amp[e];
      v = a.x * a.x + a.y * a.y;
    }
    head = 1;
    if (e > 0) {
      uint64_t q[W];
#pragma unroll
      for (int j = 0; j < W; ++j) q[j] = keys.w[j][e - 1];
      const uint64_t qi = f.has_inst ? ((sel_word<W>(q, f.iword) >> f.ishift) & f.imask) : 0;
      const uint64_t qv = (sel_word<W>(q, f.fword) >> f.fshift) & f.fmask;
      head = (qi != ii || qv != fv) ? 1u : 0u;
    }
  }
  __syncthreads();
  if (head) atomicMin(&s_head, threadIdx.x);
  // (value, started) pairs: (a, fa) then (b, fb) gives (fb ? b : a + b, fa | fb)
  uint32_t fl = head;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double pv = __shfl_up(v, d, 64);
    const uint32_t pf = __shfl_up(fl, d, 64);
    if (lane >= (uint32_t)d) {
      if (!fl) v = pv + v;
      fl |= pf;
    }
  }
  if (lane == 63) {
    s_v[wv] = v;
    s_f[wv] = fl;
  }
  __syncthreads();
  double cv = 0.0;
  for (uint32_t j = 0; j < wv; ++j) cv = s_f[j] ? s_v[j] : cv + s_v[j];
  if (wv > 0 && !fl) v = cv + v;
  if (e < n) part[e] = v;
  const uint64_t last = ((uint64_t)blockIdx.x + 1) * kBlock < n ? ((uint64_t)blockIdx.x + 1) * kBlock - 1 : n - 1;
  if (e == last) tail[blockIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) fhead[blockIdx.x] = s_head;
}

// Sum carried into each tile by the segment that started before it (one
// thread, tiles in order).
static __global__ void k_runs_carry(const uint32_t* __restrict__ fhead, const double* __restrict__ tail,
                                    uint64_t ntiles, double* __restrict__ carry) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double c = 0.0;
  for (uint64_t t = 0; t < ntiles; ++t) {
    carry[t] = c;
    c = fhead[t] < (uint32_t)kBlock ? tail[t] : c + tail[t];
  }
}

// Each entry of the instance that ends its field's run writes the field value
// and p(v) / P (in place of its part sum); every other entry writes -1.
template <int W>
__global__ __launch_bounds__(kBlock) void k_runs_out(KeyPtrs<W> keys, uint64_t n, FilterOp f,
                                                     double* __restrict__ part, const uint32_t* __restrict__ fhead,
                                                     const double* __restrict__ carry, const double* __restrict__ total,
                                                     uint64_t* __restrict__ out_val) {
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  uint64_t k[W];
#pragma unroll
  for (int j = 0; j < W; ++j) k[j] = keys.w[j][e];
  const uint64_t ii = f.has_inst ? ((sel_word<W>(k, f.iword) >> f.ishift) & f.imask) : 0;
  const uint64_t fv = (sel_word<W>(k, f.fword) >> f.fshift) & f.fmask;
  bool end = true;
  if (e + 1 < n) {
    uint64_t q[W];
#pragma unroll
    for (int j = 0; j < W; ++j) q[j] = keys.w[j][e + 1];
    const uint64_t qi = f.has_inst ? ((sel_word<W>(q, f.iword) >> f.ishift) & f.imask) : 0;
    const uint64_t qv = (sel_word<W>(q, f.fword) >> f.fshift) & f.fmask;
    end = qi != ii || qv != fv;
  }
  const double v = part[e];
  double out = -1.0;
  if (end && (!f.has_inst || ii == f.inst)) {
    const uint32_t pos = threadIdx.x;
    const double sum = pos < fhead[blockIdx.x] ? carry[blockIdx.x] + v : v;
    out = sum / *total;
    out_val[e] = fv;
  }
  part[e] = out;
}

// Copy n entries between buffers of key widths WI <= WO (words WI.. of the
// output are 0): re-packing for keys that gain words.
template <int WI, int WO>
__global__ __launch_bounds__(kBlock) void k_relayout(KeyPtrs<WI> in_keys, const double2* __restrict__ in_amp,
                                                     KeyPtrs<WO> out_keys, double2* __restrict__ out_amp, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int w = 0; w < WO; ++w) out_keys.w[w][i] = w < WI ? in_keys.w[w < WI ? w : 0][i] : 0ull;
    out_amp[i] = in_amp[i];
  }
}

}  // namespace sparqs
