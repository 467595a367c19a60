// Internal structures shared by the host planner and the gfx950 kernels of
// the sparse register-level simulator.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sparqs {

constexpr int kMaxW = 4;            // 64-bit key words per entry (up to 256 key bits)
constexpr int kBlock = 256;         // threads per workgroup (4 wave64)
constexpr int kRadixBits = 8;       // digit width of one radix-sort pass
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxFields = 8;       // contiguous bit runs that make up one digit
constexpr int kMaxPasses = 40;      // up to 256 key bits + 5 target bits, 8 bits per pass
constexpr int kMaxGroupBits = 5;    // targets fused into one interference op (2^5 group)
constexpr int kMaxExpandBits = 10;  // targets of one pure expansion (one thread per child, 2^10 children)
constexpr int kRing = 128;          // per-launch slots (tile counter, count, key masks)
constexpr int kBaseGens = 64;       // retirement generations kept in the meta block (batched rounds)
constexpr int kXcds = 8;            // XCDs of an MI355X
constexpr uint32_t kTileChunk = 8;  // consecutive tiles per XCD with chunked tickets
constexpr int kXcdStride = 16;      // per-XCD counters 128 bytes apart

// Lookback words: [epoch:24 | flag:2 | value:38].
constexpr uint64_t kLbValueBits = 38;
constexpr uint64_t kLbValueMask = (1ull << kLbValueBits) - 1;
constexpr uint64_t kLbAgg = 1ull << kLbValueBits;
constexpr uint64_t kLbInc = 2ull << kLbValueBits;
constexpr uint64_t kLbFlagMask = 3ull << kLbValueBits;
constexpr int kLbEpochShift = 40;
constexpr uint32_t kEpochMask = (1u << 24) - 1;

// Error bits raised by kernels (meta->err).
constexpr uint32_t kErrCapacity = 1u << 0;   // outputs would exceed the buffer capacity
constexpr uint32_t kErrSpin = 1u << 1;       // a lookback wait exceeded its bound
constexpr uint32_t kErrGroup = 1u << 2;      // two group members share a target value
constexpr uint32_t kErrGrid = 1u << 3;       // a grid was sized below the entry count (host bug)
constexpr uint32_t kErrPlan = 1u << 4;       // a graph replay met a count or key mask its plan did not
// After a speculative fixed-placement launch is wasted, this many eligible
// ops of the same mode (group or expand) skip speculation (on the device
// until the next read-back, then on the host); a skipped launch leaves
// kSpecSkipped in its flag.
constexpr uint32_t kSpecCool = 64;
constexpr unsigned int kSpecSkipped = 2u;

// Device-side bookkeeping.  Every kernel launch that counts tiles, produces an
// entry count or key masks owns ring slot (epoch % kRing); workgroup 0 of
// launch e clears slot (e + kRing/2) % kRing for a later launch.  The host
// reads back the leading status part (up to `dscratch`) when it synchronises.
struct DevMeta {
  unsigned long long nring[2];               // entry count: launches read one slot, emitters write the other
  unsigned long long peak;                   // running maximum of nnz
  unsigned int err;                          // kErr* bits, sticky until the host clears them
  unsigned int err_epoch;                    // epoch of the launch that raised the first error
  unsigned long long upd;                    // entries updated: sum over ops of the input count
  unsigned long long spec_fail[2];           // speculative launches that met an irregular tile, per mode
  unsigned long long nnz_out[kRing];         // entry count written by an emitting kernel
  unsigned long long or_mask[kRing][kMaxW];  // OR of the produced keys, per word
  unsigned long long and_mask[kRing][kMaxW]; // AND of the produced keys, per word
  unsigned long long base_gen[kBaseGens];    // retired prefix per retirement generation (batched rounds)
  // device-only part
  double dscratch[16];
  unsigned long long uscratch[16];
  unsigned long long counters[kRing];        // dynamic tile ids (one ticket per launch)
  unsigned int spec_irr[kRing];              // speculative launch: 1 met an irregular tile, kSpecSkipped skipped
  unsigned int spec_cool[2];                 // speculative launches left to skip after a wasted one, per mode
  unsigned long long xcd_ctr[kRing][kXcds * kXcdStride];  // per-XCD tickets
  // Batched rounds retire finished instances: entries [0, base) of both
  // entry buffers are final and the round kernels (and the sort) work on the
  // view [base, n).  0 outside batched rounds.
  unsigned long long base;
  unsigned long long retire_p;               // end of the next retired block (set by k_retire_copy)
};

// A run of non-branching ops is executed from an array of these (uniform per op).
// Field positions are precomputed on the host; `dst_*` is the written register,
// `src_*` the read register (ADD/SUB/XOR source, QRAM address).
enum PermKind : uint32_t {
  PK_XMASK = 0,     // key[w] ^= imm (the qubit mask, shifted) on dst word
  PK_ADD = 1,
  PK_SUB = 2,
  PK_MULC = 3,
  PK_XOR = 4,
  PK_XORC = 5,      // same as XMASK but kept distinct for statistics
  PK_QRAM = 6,
  PK_REFLECT0 = 7,
  PK_DIAG = 8,      // per qubit of imm (shifted, ascending): amplitude *= fac[bit]
  PK_ADIAG = 9,     // the same, then the qubits of imm flip
  PK_ADDC = 10,     // dst += imm
  PK_MUL = 11,      // dst ^= src * src2
  PK_DIV = 12,      // dst ^= src div src2, dst2 ^= src mod src2
};

struct PermOp {
  uint32_t kind;
  uint32_t nctl_words;          // 0: uncontrolled
  uint32_t dst_word, dst_shift;
  uint32_t src_word, src_shift;
  uint32_t table_words32;       // 1 if the QRAM table is stored as uint32
  uint32_t pad;
  uint64_t dst_mask;            // (1 << width) - 1, unshifted
  uint64_t src_mask;
  uint64_t imm;                 // X mask / XOR constant / multiplier (already shifted for X)
  const void* table;            // QRAM words
  uint64_t cmask[kMaxW];        // control bits per word
  uint64_t cval[kMaxW];         // required values of those bits
  uint32_t src2_word, src2_shift;  // MUL second factor / DIV divisor
  uint32_t dst2_word, dst2_shift;  // DIV remainder
  uint64_t src2_mask, dst2_mask;
  double fac[2][2];             // PK_DIAG / PK_ADIAG: factor (re, im) for input bit 0 and 1
};

// Fast form of a non-branching op for keys of at most 2 words, every field
// inside one 32-bit half of a word (halves numbered word*2 + upper).  `code`
// fixes the op kind and the half indices, so each case of the interpreter is
// straight-line code on named registers.
enum FastBase : uint32_t {
  F_XM = 0,       // + h          : h ^= imm                     (X / XORC, uncontrolled)
  F_XC1 = 4,      // + t*4 + c    : h[t] ^= imm if bit cb of h[c] is 1      (CNOT)
  F_XC1N = 20,    // + t*4 + c    : h[t] ^= imm if bit cb of h[c] is 0
  F_XC2 = 36,     // + t*16+c*4+c2: two controls                            (Toffoli)
  F_ADDA = 100,   // + d*4 + s    : h[d] += h[s]   (both whole halves)
  F_ADDF = 116,   // + d*4 + s    : field form
  F_SUBA = 132,
  F_SUBF = 148,
  F_XORA = 164,
  F_XORF = 180,
  F_MULA = 196,   // + d
  F_MULF = 200,   // + d
  F_QRAM = 204,   // + d*4 + s    : data field ^= table32[address field]
  F_REFL = 220,   // + d          : amplitude *= +i / -i by field == 0
  F_GEN = 224,    // generic 64-bit form: gops[gi]
  F_NCODES = 225
};

// One record per op, 32 bytes so that a single scalar load brings it in;
// the meaning of a..f depends on the kind:
//   X / XORC:   imm = mask in place
//   one control:  a = control bit
//   two controls: a, b = control bits; c, d = all ones where that control's
//                 required value is 0
//   fields (ADD/SUB/XOR, MUL, QRAM, REFL): a = destination shift, b =
//                 destination mask in place, c = source shift, d = source bits
//                 taken (min of both widths, < 32; MUL: destination width;
//                 QRAM: address mask), imm = multiplier
//   QRAM: e, f = table address (low, high word);  generic: e = record index
struct alignas(32) FastOp {
  uint32_t code, imm;
  uint32_t a, b, c, d, e, f;
};
static_assert(sizeof(FastOp) == 32, "one 32-byte record per op");

constexpr int kMaxChain = 16;       // one-target ops on one target fused into one launch

// One op of a chain: its real 2x2 matrix (m[out][in]) and its controls
// (cmask 0: uncontrolled).  The controls never include the target bit, so
// both members of a group see the same ones.
struct ChainStep {
  double m[2][2];
  uint64_t cmask[kMaxW];
  uint64_t cval[kMaxW];
};

// One branching (interference) op as seen by the group/expand kernel.
struct GroupOp {
  uint32_t k;                   // target qubits (1..kMaxGroupBits; up to kMaxExpandBits in expand mode)
  uint32_t has_ctl;
  uint32_t upd;                 // ops to count: the update counter gains upd x the input count
  uint32_t nchain;              // k == 1 only: > 0 applies chain[0..nchain) (m, cmask, cval unused)
  const ChainStep* chain;       // device array
  uint32_t tword[kMaxExpandBits];  // target j: key word and bit, ascending qubit order
  uint32_t tbit[kMaxExpandBits];
  uint64_t tmask[kMaxW];        // all target bits per word
  uint64_t cmask[kMaxW];
  uint64_t cval[kMaxW];
  double m[2][2];               // matrix, m[out][in] (real parts)
  double eps2;                  // prune below this |a|^2 (strict)
  uint32_t cplx;                // 1: mi holds imaginary parts (k == 1, no chain)
  uint32_t pad;
  double mi[2][2];
};

// Key bits a captured plan allows to vary at one of its check points.
struct PlanVar {
  uint64_t var[kMaxW];
};

// Per-instance tables of a batched round (instances with their own op lists).
struct RunRange {
  uint32_t start, len;          // FastOp range of the instance's non-branching run
};

struct alignas(16) BatchOp {     // staged in LDS as 16-byte words
  uint32_t k;                   // target qubits this round (0: the entry passes through)
  uint32_t has_ctl;
  uint32_t prune;               // 1: the instance branched this round; apply eps2 after merging
  uint32_t pad;
  uint32_t tword[kMaxGroupBits], tbit[kMaxGroupBits];
  uint64_t cmask[kMaxW], cval[kMaxW];
  double m[2][2];
  double eps2;
  uint32_t cplx;                // 1: mi holds imaginary parts (k == 1)
  uint32_t pad2;
  double mi[2][2];
};
static_assert(sizeof(BatchOp) % 16 == 0, "BatchOp is staged as 16-byte words");

// A digit of one radix pass = sum of up to kMaxFields bit runs of the key:
//   digit |= ((key[word] >> shift) & ((1 << width) - 1)) << dshift
struct PassDesc {
  uint32_t nf;
  uint32_t f[kMaxFields];       // word:2 | shift:6 | width:4 | dshift:4  (packed)
};

__host__ __device__ inline uint32_t pack_field(uint32_t word, uint32_t shift, uint32_t width,
                                               uint32_t dshift) {
  return word | (shift << 2) | (width << 8) | (dshift << 12);
}

struct SortPlan {
  uint32_t npass;
  PassDesc pass[kMaxPasses];
};

}  // namespace sparqs
