// C ABI and host planner of the sparse register-level simulator (one MI355X).
//
// The planner turns a list of register-level ops into kernel launches:
//  * consecutive non-branching ops form one fused k_perm launch;
//  * a branching op (H / Ry on up to 5 qubits per launch) becomes
//      - k_group in EXPAND mode when none of its target bits varies over the
//        state (every group has one member),
//      - k_group in GROUP mode directly when the entries are still grouped by
//        the same target bits (members of a group contiguous), which the
//        planner tracks through ops that cannot separate group members,
//      - otherwise an LSD radix sort on (idle bits that vary, target bits)
//        followed by k_group.
// Control reaches the device once per launch; the host reads back the entry
// count and key masks after each branching op (a pinned 2 KB block).
#include "../../include/sparqs.h"
#include "kernels.hip"
#include "launch.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace sparqs;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint32_t kMaxOpsPerCall = 16384;  // device op ring, in PermOp records
constexpr uint64_t kOpRingBytes = (uint64_t)kMaxOpsPerCall * sizeof(PermOp);
constexpr uint32_t kRunChunk = 4096;        // ops per fused launch
constexpr uint64_t kUploadOps = 256;        // non-branching ops whose records one copy uploads
constexpr uint64_t kSmallSort = 1ull << 16; // at most this many entries: sort plans from the host superset
constexpr uint32_t kHistBlocksMax = 16384;  // further bounded by kHistWaves x the resident count
constexpr uint32_t kHistWaves = 2;         // histogram workgroups per resident slot

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct RegInfo {
  uint32_t word, shift, width;
  uint64_t mask;
};

struct TableInfo {
  void* dev;
  uint32_t addr_bits, word_bits;
  bool w32;
};

// A 2x2 complex matrix, m[out][in] as (re, im).
struct Mat2 {
  double re[2][2], im[2][2];
};

struct Layout {
  std::vector<RegInfo> regs;
  uint32_t W = 1;
  bool has_inst = false;
  uint32_t iword = 0, ishift = 0, ibits = 0;
  uint64_t imask = 0;
};

int make_layout(const ss_reg* regs, uint32_t nregs, uint32_t ninst, Layout& L) {
  if (!regs || nregs == 0 || nregs > 64 || ninst == 0) return SS_E_ARG;
  uint32_t fill[kMaxW] = {0, 0, 0, 0};
  uint32_t used = 0;
  auto place = [&](uint32_t width, uint32_t& word, uint32_t& shift) -> bool {
    for (uint32_t w = 0; w < (uint32_t)kMaxW; ++w) {
      if (fill[w] + width <= 64) {
        word = w;
        shift = fill[w];
        fill[w] += width;
        used = std::max(used, w + 1);
        return true;
      }
    }
    return false;
  };
  L.regs.clear();
  for (uint32_t r = 0; r < nregs; ++r) {
    const uint32_t w = regs[r].nqubits;
    if (w < 1 || w > 64) return SS_E_ARG;
    RegInfo ri;
    if (!place(w, ri.word, ri.shift)) return SS_E_ARG;
    ri.width = w;
    ri.mask = w == 64 ? ~0ull : ((1ull << w) - 1);
    L.regs.push_back(ri);
  }
  L.has_inst = ninst > 1;
  if (L.has_inst) {
    uint32_t b = 0;
    while ((1ull << b) < ninst) ++b;
    L.ibits = b;
    L.imask = (1ull << b) - 1;
    if (!place(b, L.iword, L.ishift)) return SS_E_ARG;
  }
  L.W = used <= 1 ? 1 : (used <= 2 ? 2 : 4);
  return SS_OK;
}

uint64_t entry_bytes(uint32_t W) { return 8ull * W + 16; }

struct Carve {
  uint64_t meta, digit_start, dev_ops, uscr, hist, tables, lb, buf0, buf1, total;
  uint64_t lb_words, hist_blocks;
};

// Radix passes a sort of W-word keys can need: every key bit plus the
// targets of one interference op, 8 bits per pass.
uint64_t max_passes(uint32_t W) { return (64ull * W + kMaxGroupBits + kRadixBits - 1) / kRadixBits; }

Carve carve(uint32_t W, uint32_t ninst, uint64_t cap, uint64_t table_bytes) {
  Carve c{};
  uint64_t off = 0;
  c.meta = off;
  off = align_up(off + sizeof(DevMeta), kAlign);
  c.digit_start = off;
  off = align_up(off + (uint64_t)kMaxPasses * kRadix * 8, kAlign);
  c.dev_ops = off;
  off = align_up(off + (uint64_t)kMaxOpsPerCall * sizeof(PermOp), kAlign);
  c.uscr = off;
  off = align_up(off + (uint64_t)(ninst + 64) * 8, kAlign);
  // the tables' place does not depend on the key width (a key that gains
  // words re-carves the arena around them)
  c.tables = off;
  off = align_up(off + table_bytes, kAlign);
  c.hist_blocks = std::min<uint64_t>(kHistBlocksMax, std::max<uint64_t>(1, cap / 4096));
  c.hist = off;
  off = align_up(off + max_passes(W) * kRadix * 8, kAlign);
  // look-back words: sort tiles (>= 2048 entries) x 256 digits, emit tiles (256 entries)
  c.lb_words = std::max<uint64_t>(cap / 2048 + 2, 1) * kRadix + cap / kBlock + 64;
  c.lb = off;
  off = align_up(off + c.lb_words * 8, kAlign);
  c.buf0 = off;
  off = align_up(off + cap * entry_bytes(W), kAlign);
  c.buf1 = off;
  off = align_up(off + cap * entry_bytes(W), kAlign);
  c.total = off;
  return c;
}

}  // namespace

struct ss_state {
  Layout L;
  uint32_t ninst = 1;
  double eps = 0.0;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  uint64_t table_bytes = 0;
  uint64_t cap = 0;
  Carve cv{};
  Buf buf[2]{};
  int cur = 0;
  DevMeta* meta = nullptr;
  uint64_t* lb = nullptr;
  unsigned long long* hist = nullptr;   // global digit counts, one histogram per pass
  uint64_t* digit_start = nullptr;
  PermOp* dev_ops = nullptr;
  uint64_t* uscr = nullptr;
  char* tab_base = nullptr;
  uint64_t tab_used = 0;
  std::vector<TableInfo> tables;
  std::vector<Mat2> mats;         // ROT matrices (ss_load_matrix)
  // Host view of the entry count.  The count itself lives on the device in
  // meta->nring[nslot]: an emitting launch reads slot nslot and writes the
  // other one.  Between synchronisations the host knows an upper bound only.
  uint32_t nslot = 0;
  uint64_t n = 0;                 // exact count (valid when n_known)
  bool n_known = true;
  uint64_t n_ub = 0;              // upper bound of the count (== n when known)
  // estimate of the count for launch heuristics: exact at read-backs, times
  // 2^k per expansion, kept by group ops (which grow only where a member
  // without its partner meets a mixing matrix) and by compactions
  uint64_t n_est = 0;
  uint32_t n_src_ep = 0;          // launch whose output count is current (0: n is exact)
  uint64_t peak = 0;
  // key masks: OR / AND over all keys, per word
  uint64_t orm[kMaxW]{}, andm[kMaxW]{};
  bool masks_valid = false;       // orm/andm describe the current entries
  // A superset of the varying key bits kept on the host without read-backs:
  // a key bit clear in sorm is 0 in every entry, one set in sandm is 1 in
  // every entry.  Updated per op from what the op can write; exact whenever
  // exact masks are read back.  It decides expansions (target bits provably
  // constant) without a synchronisation; sorts still use exact masks.
  uint64_t sorm[kMaxW]{}, sandm[kMaxW]{};
  bool sup_valid = false;
  uint32_t mask_ep = 0;           // launch whose ring slot holds them (0: none, recompute)
  uint32_t epoch = 0;
  bool grouped = false;
  uint64_t gmask[kMaxW]{};
  bool poisoned = false;
  // capacity-checked launches since the last synchronisation, for rollback
  struct EmitLog {
    uint32_t ep;
    int cur;
    uint32_t nslot;
    uint64_t op;
  };
  std::vector<EmitLog> emits;
  // Graph capture (ss_graph_capture).  The planner runs the op list once for
  // real while recording every read-back of the status block, then once more
  // under stream capture, where each synchronisation takes the recorded
  // read-back instead and enqueues a check kernel: a replay must meet the same
  // entry count there and no key bit varying that did not vary then.
  enum { G_EAGER = 0, G_RECORD = 1, G_CAPTURE = 2 };
  int gmode = G_EAGER;
  std::vector<std::vector<char>> snaps;
  size_t snap_pos = 0;
  uint64_t rec_bytes = 0;         // op-record bytes the recording run uploaded
  char* cap_hops = nullptr;       // graph-owned pinned op records (capture)
  uint64_t cap_used = 0, cap_size = 0;
  bool final_sync = false;        // the synchronisation that ends a call: no check
  // last consistent point (buffer, count slot, op or round index) and the
  // buffer swaps since: a check can roll back to it while at most one swap
  // (one emitting launch) has happened, i.e. its buffer is still intact
  struct PlanMark {
    uint32_t ep;
    int cur;
    uint32_t nslot;
    uint64_t op;
    bool valid;
  };
  PlanMark mark{};
  uint32_t flips = 0;
  std::vector<PlanMark> plan_log;  // check points of a replay, for rollback
  std::vector<ss_graph*> graphs;   // live graphs built on this state
  bool rolled_back = false;       // the last synchronisation rolled back a launch
  uint64_t rb_op = 0;             // ... whose op index (batched: round) this is
  uint32_t dev_err = 0;           // kernel-side error bits seen at the last read-back
  bool static_scratch = false;    // scratch in the library's device array (ss_create_state_noalloc)
  int static_dev = -1;            // ... of this device
  DevMeta* hmeta = nullptr;       // pinned read-back block
  PermOp* hops = nullptr;         // pinned op staging (kMaxOpsPerCall)
  uint32_t ops_used = 0;
  // bytes at the start of the op ring that hold records uploaded for launches
  // not made yet: a synchronisation frees the ring only above them
  uint32_t ops_keep = 0;
  // options
  int sort_items = 16;
  int grouping = 1;
  int group_items = 4;
  int perm_entries = 8;
  // option: a one-target expansion on at least this many entries (upper
  // bound) first tries the fixed-fan-out placement; 0 never.  Below a few
  // million entries the look-back chain is short and the extra launch costs
  // more than it saves.
  uint64_t speculate = 1ull << 23;
  // option: the same for one-target ops on grouped entries (0: never).  There
  // a merge (destructive interference) or a member without its partner
  // leaves the fixed placement; after a wasted launch the next kSpecCool
  // eligible launches skip themselves on the device, and once a read-back sees
  // it the host does not launch them for the next kSpecCool eligible ops (twice
  // as many each time that repeats; back to kSpecCool after a read-back that
  // finds speculative launches and none wasted).
  uint64_t spec_group = 1ull << 21;
  uint32_t spec_items = 4;       // option: entries per thread of the speculative launch (1|2|4)
  int expand_slots = 1;          // option: expansions on 2..5 targets one thread per child (0: per entry)
  uint32_t pair_exchange = 2;    // option: how speculative group launches find partners (0 | 1 | 2)
  // per mode (group, expand):
  uint64_t spec_fail_seen[2] = {0, 0};  // device count of wasted speculative launches at the last read-back
  uint32_t spec_skip[2] = {0, 0};       // eligible ops left that do not speculate
  uint32_t spec_backoff[2] = {kSpecCool, kSpecCool};  // the next skip length (doubles while wasted)
  uint32_t spec_tries[2] = {0, 0};      // speculative launches since the last read-back
  int chain = 1;                 // option: consecutive one-target ops on one target in one launch
  // option: a one-target op applies the run that follows it when the run has
  // at most this many ops (0: never); fusing saves the run's own read and
  // write of the state.
  uint32_t fuse_runs = kRunChunk;
  // batched rounds: relabel instances by the round of their last op and
  // leave the finished ones out of later rounds (option "retire")
  bool retire_batched = true;
  bool in_view = false;           // launches work on the view [base, n) (batched rounds)
  uint32_t vgen = 0;              // retirement generation of the current view base
  std::vector<uint32_t> undo_map; // instance of each label of the last batched call (empty: not relabelled)
  uint32_t xcd_order = 0;        // 1 when workgroups spread round-robin over 8 XCDs
  uint32_t hist_res[3] = {1024, 1024, 1024};  // resident k_sort_hist workgroups, W = 1, 2, 4
  int tile_order_opt = 1;        // option: 1 use XCD tickets when possible, 0 one counter
  uint64_t stats[8]{};
  // per-launch HIP-event timing (option "trace")
  bool trace = false;
  std::vector<hipEvent_t> ev_pool;
  // Bytes and entries of a traced launch depend on counts that the host
  // learns at the next synchronisation: input count n_in (exact, or the
  // output of launch in_ep), output count (of launch out_ep, if it emits).
  struct TraceRec {
    uint32_t cat;
    hipEvent_t a, b;
    uint32_t in_ep, out_ep;
    uint64_t in_n, in_per, out_per, ent_mult;
    int64_t vgen;                 // >= 0: counts are of the view past that generation's base
  };
  std::vector<TraceRec> pending;
  uint32_t trace_old_ep = 0;      // oldest launch a pending record refers to
  double tr_sec[SS_TRACE_NCAT]{};
  uint64_t tr_cnt[SS_TRACE_NCAT]{}, tr_bytes[SS_TRACE_NCAT]{}, tr_entries[SS_TRACE_NCAT]{};
};

namespace {

Buf make_buf(char* base, uint32_t W, uint64_t cap) {
  Buf b{};
  for (uint32_t w = 0; w < W; ++w) b.key[w] = reinterpret_cast<uint64_t*>(base + (uint64_t)w * cap * 8);
  b.amp = reinterpret_cast<double2*>(base + (uint64_t)W * cap * 8);
  return b;
}

template <int W>
KeyPtrs<W> kp(const Buf& b) {
  KeyPtrs<W> p;
  for (int w = 0; w < W; ++w) p.w[w] = b.key[w];
  return p;
}

int hip_fail(ss_state* st) {
  st->poisoned = true;
  return SS_E_HIP;
}

uint32_t xo(const ss_state* st) { return (st->xcd_order && st->tile_order_opt) ? 1u : 0u; }

// Launch context: read buf[cur], write buf[cur ^ 1].
LaunchCtx ctx(const ss_state* st) {
  LaunchCtx c;
  c.stream = st->stream;
  c.in = st->buf[st->cur];
  c.out = st->buf[st->cur ^ 1];
  c.ns = st->nslot;
  c.cap = st->cap;
  c.n_ub = st->n_ub;
  c.lb = st->lb;
  c.meta = st->meta;
  c.xo = xo(st);
  return c;
}

int check_launch(ss_state* st) {
  if (hipGetLastError() != hipSuccess) return hip_fail(st);
  return SS_OK;
}

// Event pair around one launch when tracing; returns the record index or -1.
int trace_begin(ss_state* st, uint32_t cat) {
  if (!st->trace) return -1;
  hipEvent_t ev[2];
  for (int i = 0; i < 2; ++i) {
    if (!st->ev_pool.empty()) {
      ev[i] = st->ev_pool.back();
      st->ev_pool.pop_back();
    } else if (hipEventCreate(&ev[i]) != hipSuccess) {
      return -1;
    }
  }
  (void)hipEventRecord(ev[0], st->stream);
  ss_state::TraceRec r{};
  r.cat = cat;
  r.a = ev[0];
  r.b = ev[1];
  st->pending.push_back(r);
  return (int)st->pending.size() - 1;
}

// Close a record: input bytes/entries per input entry, output bytes per
// output entry of the emitting launch `out_ep` (0: none).
void trace_end(ss_state* st, int idx, uint64_t in_per, uint64_t ent_mult, uint32_t out_ep, uint64_t out_per) {
  if (idx < 0) return;
  auto& r = st->pending[(size_t)idx];
  r.in_ep = st->n_src_ep;
  r.in_n = st->n;
  r.in_per = in_per;
  r.ent_mult = ent_mult;
  r.out_ep = out_ep;
  r.out_per = out_per;
  r.vgen = st->in_view ? (int64_t)st->vgen : -1;
  for (uint32_t e : {r.in_ep, r.out_ep})
    if (e && (st->trace_old_ep == 0 || e < st->trace_old_ep)) st->trace_old_ep = e;
  (void)hipEventRecord(r.b, st->stream);
}

// After a read-back of the meta block: fold finished records into the totals.
void trace_flush(ss_state* st) {
  const DevMeta* hm = st->hmeta;
  for (auto& r : st->pending) {
    float ms = 0.f;
    uint64_t n_in = r.in_ep ? hm->nnz_out[r.in_ep % kRing] : r.in_n;
    uint64_t n_out = r.out_ep ? hm->nnz_out[r.out_ep % kRing] : 0;
    if (r.vgen >= 0) {
      // batched rounds: only the entries past the retired prefix were touched
      const uint64_t b = hm->base_gen[r.vgen % kBaseGens];
      n_in = n_in > b ? n_in - b : 0;
      n_out = n_out > b ? n_out - b : 0;
    }
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      st->tr_sec[r.cat] += ms * 1e-3;
      st->tr_cnt[r.cat] += 1;
      st->tr_bytes[r.cat] += n_in * r.in_per + n_out * r.out_per;
      st->tr_entries[r.cat] += n_in * r.ent_mult;
    }
    st->ev_pool.push_back(r.a);
    st->ev_pool.push_back(r.b);
  }
  st->pending.clear();
  st->trace_old_ep = 0;
}

void drop_trace(ss_state* st) {
  for (auto& r : st->pending) {
    st->ev_pool.push_back(r.a);
    st->ev_pool.push_back(r.b);
  }
  st->pending.clear();
  st->trace_old_ep = 0;
}

void take_masks(ss_state* st, uint32_t ep) {
  const uint32_t r = ep % kRing;
  for (int w = 0; w < kMaxW; ++w) {
    st->orm[w] = st->sorm[w] = st->hmeta->or_mask[r][w];
    st->andm[w] = st->sandm[w] = st->hmeta->and_mask[r][w];
  }
  st->masks_valid = true;
  st->sup_valid = true;
}

// The superset after an op that may set `bits` of `word` to anything.
// Shape of a ROT matrix: 1 diagonal, 2 off-diagonal (each branch stays one
// branch), 0 general.  An element is zero when both its parts are 0.0.
int mat_shape(const Mat2& m) {
  auto zero = [&](int r, int c) { return m.re[r][c] == 0.0 && m.im[r][c] == 0.0; };
  if (zero(0, 1) && zero(1, 0)) return 1;
  if (zero(0, 0) && zero(1, 1)) return 2;
  return 0;
}

// Interference (branching) ops: H, Ry and a rotation by a general matrix.
bool is_branching(const ss_state* st, const ss_op& op) {
  if (op.kind == SS_H || op.kind == SS_RY) return true;
  return op.kind == SS_ROT && op.aux < st->mats.size() && mat_shape(st->mats[op.aux]) == 0;
}

// The one-to-one single-qubit gates: a key bit flip (off-diagonal) or not,
// and the factor taking input bit b to its output bit.
bool one_to_one(const ss_state* st, const ss_op& op, bool* flip, double (&fac)[2][2]) {
  const double c = 0.70710678118654752440;  // cos(pi/4) = sin(pi/4) as the nearest double
  fac[0][0] = 1.0; fac[0][1] = 0.0; fac[1][0] = 1.0; fac[1][1] = 0.0;
  *flip = false;
  switch (op.kind) {
    case SS_Y: *flip = true; fac[0][0] = 0.0; fac[0][1] = 1.0; fac[1][0] = 0.0; fac[1][1] = -1.0; return true;
    case SS_Z: fac[1][0] = -1.0; return true;
    case SS_S: fac[1][0] = 0.0; fac[1][1] = 1.0; return true;
    case SS_SDG: fac[1][0] = 0.0; fac[1][1] = -1.0; return true;
    case SS_T: fac[1][0] = c; fac[1][1] = c; return true;
    case SS_TDG: fac[1][0] = c; fac[1][1] = -c; return true;
    case SS_PHASE: fac[1][0] = std::cos(op.theta); fac[1][1] = std::sin(op.theta); return true;
    case SS_ROT: {
      if (op.aux >= st->mats.size()) return false;
      const Mat2& m = st->mats[op.aux];
      const int sh = mat_shape(m);
      if (sh == 0) return false;
      // diagonal: bit b keeps, factor m[b][b]; off-diagonal: factor m[1-b][b]
      for (int b = 0; b < 2; ++b) {
        const int r = sh == 1 ? b : 1 - b;
        fac[b][0] = m.re[r][b];
        fac[b][1] = m.im[r][b];
      }
      *flip = sh == 2;
      return true;
    }
    default:
      return false;
  }
}

// Whether a non-branching op changes amplitudes, and the key words it writes.
bool op_uses_amp(const ss_state* st, const ss_op& op) {
  bool flip;
  double fac[2][2];
  return op.kind == SS_REFLECT0 || one_to_one(st, op, &flip, fac);
}

uint32_t op_write_words(const ss_state* st, const ss_op& op) {
  bool flip;
  double fac[2][2];
  if (op.kind == SS_REFLECT0) return 0;
  if (one_to_one(st, op, &flip, fac) && !flip) return 0;
  uint32_t ww = 1u << st->L.regs[op.reg].word;
  if (op.kind == SS_DIV) ww |= 1u << st->L.regs[op.imm].word;
  return ww;
}

void sup_vary(ss_state* st, uint32_t word, uint64_t bits) {
  st->sorm[word] |= bits;
  st->sandm[word] &= ~bits;
}

// ... after an op that flips `bits` of `word` in every entry.
void sup_flip(ss_state* st, uint32_t word, uint64_t bits) {
  const uint64_t o = st->sorm[word], a = st->sandm[word];
  st->sorm[word] = (o & ~bits) | (~a & bits);
  st->sandm[word] = (a & ~bits) | (~o & bits);
}

// ... after a non-branching op.
void sup_op(ss_state* st, const ss_op& op) {
  const RegInfo& d = st->L.regs[op.reg];
  bool flip;
  double fac[2][2];
  if (one_to_one(st, op, &flip, fac)) {
    // keys unchanged, or the mask bits flipped like X
    if (flip) {
      const uint64_t bits = (op.qmask & d.mask) << d.shift;
      if (op.nctl == 0) sup_flip(st, d.word, bits);
      else sup_vary(st, d.word, bits);
    }
    return;
  }
  switch (op.kind) {
    case SS_REFLECT0:
      break;
    case SS_DIV: {
      const RegInfo& r = st->L.regs[op.imm];
      sup_vary(st, d.word, d.mask << d.shift);
      sup_vary(st, r.word, r.mask << r.shift);
      break;
    }
    case SS_X:
    case SS_XORC: {
      const uint64_t bits = ((op.kind == SS_X ? op.qmask : op.imm) & d.mask) << d.shift;
      if (op.nctl == 0) sup_flip(st, d.word, bits);
      else sup_vary(st, d.word, bits);
      break;
    }
    default:
      sup_vary(st, d.word, d.mask << d.shift);
      break;
  }
}

void set_known(ss_state* st, uint64_t n) {
  st->n = n;
  st->n_known = true;
  st->n_ub = n;
  st->n_est = n;
  st->n_src_ep = 0;
}

// Synchronise: wait for the stream, copy the status part of the device meta
// block to pinned memory and bring the host view up to date.  A launch that
// ran out of capacity made every later launch a no-op; the state returns to
// that launch's input (buffer and count), and SS_E_CAPACITY is returned with
// rolled_back / rb_op set.  Any other kernel-side error poisons the state.
void set_mark(ss_state* st, uint64_t op, bool valid = true) {
  st->mark = {0u, st->cur, st->nslot, op, valid};
  st->flips = 0;
}

void roll_back(ss_state* st, int cur, uint32_t nslot, uint64_t op) {
  st->cur = cur;
  st->nslot = nslot;
  st->rb_op = op;
  st->rolled_back = true;
  set_known(st, st->hmeta->nring[nslot]);
  st->masks_valid = false;
  st->sup_valid = false;
  st->mask_ep = 0;
  st->grouped = false;
  st->emits.clear();
  st->plan_log.clear();
}

// Synchronise: wait for the stream, copy the status part of the device meta
// block to pinned memory and bring the host view up to date.  A launch that
// ran out of capacity made every later launch a no-op; the state returns to
// that launch's input (buffer and count), and SS_E_CAPACITY is returned with
// rolled_back / rb_op set.  A failed check of a replayed graph returns
// SS_E_PLAN the same way (rolled back to the op where the plan diverged).  Any
// other kernel-side error poisons the state.
int sync_state(ss_state* st) {
  st->rolled_back = false;
  if (st->poisoned) return SS_E_STATE;
  constexpr size_t kStatus = offsetof(DevMeta, dscratch);
  if (st->gmode == ss_state::G_CAPTURE) {
    // the read-back the recording run made at this point
    if (st->snap_pos >= st->snaps.size()) return hip_fail(st);
    std::memcpy(st->hmeta, st->snaps[st->snap_pos++].data(), kStatus);
  } else {
    if (hipMemcpyAsync(st->hmeta, st->meta, kStatus, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
        hipStreamSynchronize(st->stream) != hipSuccess)
      return hip_fail(st);
    st->stats[6]++;
    if (st->gmode == ss_state::G_RECORD) {
      const char* p = reinterpret_cast<const char*>(st->hmeta);
      st->snaps.emplace_back(p, p + kStatus);
    }
  }
  st->ops_used = st->ops_keep;
  const DevMeta* hm = st->hmeta;
  st->dev_err |= hm->err;
  trace_flush(st);
  st->peak = hm->peak;
  st->stats[7] = hm->upd;
  for (int md = 0; md < 2; ++md) {
    if (hm->spec_fail[md] != st->spec_fail_seen[md]) {
      // wasted speculation since the last read-back: skip it for a while,
      // twice as long each time this repeats
      st->spec_fail_seen[md] = hm->spec_fail[md];
      st->spec_skip[md] = st->spec_backoff[md];
      st->spec_backoff[md] = std::min<uint32_t>(st->spec_backoff[md] * 2u, 1u << 20);
    } else if (st->spec_tries[md]) {
      st->spec_backoff[md] = kSpecCool;
    }
    st->spec_tries[md] = 0;
  }
  if (hm->err & ~(kErrCapacity | kErrPlan)) {
    st->emits.clear();
    st->plan_log.clear();
    return hip_fail(st);
  }
  if (hm->err & kErrPlan) {
    const ss_state::PlanMark* e = nullptr;
    for (const auto& x : st->plan_log)
      if (x.ep == hm->err_epoch) {
        e = &x;
        break;
      }
    if (!e || !e->valid) {
      // diverged inside an op split over several launches: nothing to return to
      st->emits.clear();
      st->plan_log.clear();
      st->poisoned = true;
      return SS_E_PLAN;
    }
    roll_back(st, e->cur, e->nslot, e->op);
    k_clear_err<<<1, 64, 0, st->stream>>>(st->meta);
    if (check_launch(st)) return SS_E_HIP;
    return SS_E_PLAN;
  }
  if (hm->err & kErrCapacity) {
    const ss_state::EmitLog* e = nullptr;
    for (const auto& x : st->emits)
      if (x.ep == hm->err_epoch) e = &x;
    if (!e) {
      st->emits.clear();
      st->plan_log.clear();
      return hip_fail(st);
    }
    roll_back(st, e->cur, e->nslot, e->op);
    k_clear_err<<<1, 64, 0, st->stream>>>(st->meta);
    if (check_launch(st)) return SS_E_HIP;
    return SS_E_CAPACITY;
  }
  if (st->gmode != ss_state::G_CAPTURE) {
    // (a capture keeps the logs: a replay needs all of them at its one read-back)
    st->emits.clear();
    st->plan_log.clear();
  }
  set_known(st, hm->nring[st->nslot]);
  bool took = false;
  if (!st->masks_valid && st->mask_ep && st->epoch - st->mask_ep < (uint32_t)kRing / 2) {
    take_masks(st, st->mask_ep);
    took = true;
  }
  if (st->gmode == ss_state::G_CAPTURE && !st->final_sync) {
    PlanVar v{};
    for (int w = 0; w < kMaxW; ++w) v.var[w] = st->orm[w] & ~st->andm[w];
    k_plan_guard<<<1, 64, 0, st->stream>>>(st->meta, st->nslot, st->n, took ? (int)(st->mask_ep % kRing) : -1, v,
                                           st->epoch);
    st->stats[0]++;
    st->plan_log.push_back({st->epoch, st->mark.cur, st->mark.nslot, st->mark.op, st->mark.valid && st->flips <= 1});
    if (check_launch(st)) return SS_E_HIP;
  }
  if (st->epoch >= kEpochMask - 4096) {
    // the 24-bit look-back tag is about to wrap: start over with clean words
    k_fill_u64<<<1024, 256, 0, st->stream>>>(st->lb, st->cv.lb_words, 0ull);
    k_ring_init<<<1, 64, 0, st->stream>>>(st->meta);
    st->stats[0] += 2;
    st->epoch = 0;
    st->mask_ep = 0;
    if (check_launch(st)) return SS_E_HIP;
  }
  return SS_OK;
}

// Before a launch that takes an epoch: synchronise when a pending trace
// record or the current count's source is about to leave the ring, or when
// the epoch nears its wrap (handled inside sync_state).
int begin_launch(ss_state* st, uint32_t* ep) {
  const uint32_t lim = kRing / 2 - 8;
  bool need = st->epoch >= kEpochMask - 4096;
  if (st->trace) {
    need = need || (st->trace_old_ep && st->epoch - st->trace_old_ep >= lim);
    need = need || (st->n_src_ep && st->epoch - st->n_src_ep >= lim);
  }
  if (need) {
    const int rc = sync_state(st);
    if (rc) return rc;
  }
  st->epoch++;
  st->stats[0]++;
  *ep = st->epoch;
  return SS_OK;
}

// After an emitting launch: the output is in the other buffer and slot.
// `logged`: the launch checks capacity, so a failure can roll back to here.
void after_emit(ss_state* st, uint32_t ep, uint64_t bound, bool logged, uint64_t op) {
  if (logged) st->emits.push_back({ep, st->cur, st->nslot, op});
  st->cur ^= 1;
  st->flips++;
  st->nslot ^= 1;
  st->n_known = false;
  st->n_ub = std::min(st->cap, bound);
  st->n_est = std::min(st->n_est, st->n_ub);
  st->n_src_ep = ep;
  st->masks_valid = false;
  st->mask_ep = ep;
}

int ensure_n(ss_state* st) {
  if (st->n_known) return SS_OK;
  return sync_state(st);
}

template <int W>
void launch_masks_w(ss_state* st, uint32_t ep) {
  const Buf& b = st->buf[st->cur];
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((st->n_ub + kBlock - 1) / kBlock, 2048));
  k_masks<W><<<grid, kBlock, 0, st->stream>>>(kp<W>(b), st->nslot, st->cap, st->meta, ep);
}

// Exact key masks of the current entries (synchronises unless known).
int ensure_masks(ss_state* st) {
  if (st->masks_valid) return SS_OK;
  if (st->mask_ep == 0 || st->epoch - st->mask_ep >= (uint32_t)kRing / 2 - 8) {
    uint32_t ep;
    int rc = begin_launch(st, &ep);
    if (rc) return rc;
    switch (st->L.W) {
      case 1: launch_masks_w<1>(st, ep); break;
      case 2: launch_masks_w<2>(st, ep); break;
      default: launch_masks_w<4>(st, ep); break;
    }
    rc = check_launch(st);
    if (rc) return rc;
    st->mask_ep = ep;
  }
  int rc = sync_state(st);
  if (rc) return rc;
  if (!st->masks_valid) return hip_fail(st);
  return SS_OK;
}

// ---------------------------------------------------------------------------
// sort planning: virtual key = target bits (ascending qubit order) then the
// varying idle bits from word 0 bit 0 upwards; 8 virtual bits per pass.
// ---------------------------------------------------------------------------
void build_plan(uint32_t W, const std::vector<std::pair<uint32_t, uint32_t>>& lowbits,
                const uint64_t* skip, const uint64_t* var, SortPlan& plan) {
  std::vector<std::pair<uint32_t, uint32_t>> vb = lowbits;
  for (uint32_t w = 0; w < W; ++w)
    for (uint32_t b = 0; b < 64; ++b)
      if (((var[w] & ~skip[w]) >> b) & 1ull) vb.push_back({w, b});
  plan.npass = (uint32_t)((vb.size() + kRadixBits - 1) / kRadixBits);
  for (uint32_t p = 0; p < plan.npass; ++p) {
    PassDesc& pd = plan.pass[p];
    pd.nf = 0;
    const size_t lo = (size_t)p * kRadixBits, hi = std::min(vb.size(), lo + kRadixBits);
    size_t j = lo;
    while (j < hi) {
      const uint32_t w = vb[j].first, b = vb[j].second;
      uint32_t width = 1;
      while (j + width < hi && vb[j + width].first == w && vb[j + width].second == b + width) ++width;
      pd.f[pd.nf++] = pack_field(w, b, width, (uint32_t)(j - lo));
      j += width;
    }
  }
}

template <int W>
int run_sort_w(ss_state* st, const SortPlan& plan) {
  // the kernels read the count on the device; grids come from the host's bound
  const uint64_t n = st->n_known ? st->n : st->n_ub;
  if (plan.npass == 0 || n <= 1) return SS_OK;
  if (plan.npass > max_passes(W)) return hip_fail(st);  // the histogram area is sized for this
  const int items = (W == 4) ? 8 : st->sort_items;
  const uint64_t tile = (uint64_t)kBlock * items;
  // kHistWaves workgroups per slot the device holds at once, each taking a
  // contiguous chunk: with more chunks than slots, a CU whose workgroups
  // finish early takes more of them (measured at 2^26 entries: 1x 255 /
  // 512 us, 2x 241 / 481 us, 4x 258 / 458 us for W = 1 / 2)
  const uint32_t nb = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(st->cv.hist_blocks, (n + 4095) / 4096),
                                                   st->hist_res[W == 1 ? 0 : W == 2 ? 1 : 2]);
  int tr = trace_begin(st, SS_TRACE_SORT_HIST);
  launch_sort_hist<W>(ctx(st), nb, plan, st->hist, st->digit_start);
  trace_end(st, tr, 8ull * W, 1, 0, 0);
  st->stats[0] += 2;
  const uint32_t ntiles = (uint32_t)((n + tile - 1) / tile);
  for (uint32_t p = 0; p < plan.npass; ++p) {
    uint32_t ep;
    int rc = begin_launch(st, &ep);
    if (rc) return rc;
    tr = trace_begin(st, SS_TRACE_SORT_PASS);
    launch_sort_pass<W>(ctx(st), items, ntiles, plan.pass[p], st->digit_start + p * kRadix, ep);
    trace_end(st, tr, 2 * entry_bytes(W), 1, 0, 0);
    st->cur ^= 1;
    st->flips++;
    st->stats[1]++;
  }
  st->stats[2]++;
  st->grouped = false;
  return check_launch(st);
}

// LSD sort of the current entries (count read on the device).
int run_sort(ss_state* st, const SortPlan& plan) {
  switch (st->L.W) {
    case 1: return run_sort_w<1>(st, plan);
    case 2: return run_sort_w<2>(st, plan);
    default: return run_sort_w<4>(st, plan);
  }
}

// Canonical order: every varying bit, word 0 bit 0 least significant.
int sort_canonical(ss_state* st) {
  int rc = ensure_masks(st);
  if (rc) return rc;
  uint64_t var[kMaxW], skip[kMaxW] = {0, 0, 0, 0};
  for (int w = 0; w < kMaxW; ++w) var[w] = st->orm[w] & ~st->andm[w];
  SortPlan plan;
  build_plan(st->L.W, {}, skip, var, plan);
  return run_sort(st, plan);
}

// ---------------------------------------------------------------------------
// emitting kernels (group / expand / filter): read buf[cur], write buf[cur^1]
// ---------------------------------------------------------------------------

// ep_spec != 0 (one target only): a speculative fixed-fan-out launch of that
// epoch runs first.  Group mode's speculative launch finds partners as option
// pair_exchange says.
template <int W>
void launch_group_w(ss_state* st, int mode, const GroupOp& g, uint32_t ep, uint32_t ep_spec, const FusedRun& run) {
  const LaunchCtx c = ctx(st);
  if (g.k == 1) {
    if (ep_spec) launch_spec<W>(c, mode, (int)st->spec_items, (int)st->pair_exchange, g, ep_spec, run);
    // A chained or run-carrying group-mode launch is latency-bound (a
    // product of up to 16 matrices, an interpreted run): at most 2 entries
    // per thread, for more waves per SIMD.  Expansions keep the tuned tile
    // (measured: the fused expansion of the arithmetic-heavy circuit is
    // faster at 4).
    int items = st->group_items;
    if ((g.nchain || run.n) && items > 2 && mode == MODE_GROUP) items = 2;
    // after a speculative launch the compacting one usually only records the
    // count: its cost is the dispatch of its grid, so it takes the largest tile
    if (ep_spec) items = 4;
    launch_pair<W>(c, mode, items, g, ep, ep_spec, run);
    return;
  }
  launch_multi<W>(c, mode, st->group_items, st->expand_slots != 0, g, ep);
}

template <int W>
void launch_filter_w(ss_state* st, const FilterOp& f, uint32_t ep) {
  const Buf& in = st->buf[st->cur];
  const Buf& out = st->buf[st->cur ^ 1];
  constexpr int ITEMS = 4;
  const uint32_t ntiles = ticket_grid((st->n_ub + kBlock * ITEMS - 1) / (kBlock * ITEMS), xo(st));
  k_filter<W, ITEMS><<<ntiles, kBlock, 0, st->stream>>>(kp<W>(in), in.amp, kp<W>(out), out.amp, st->nslot,
                                                        st->cap, f, st->lb, st->meta, ep, xo(st));
}

// Compaction (never grows the state); asynchronous.
int run_filter(ss_state* st, const FilterOp& f) {
  if (st->n_ub == 0) return SS_OK;
  uint32_t ep;
  int rc = begin_launch(st, &ep);
  if (rc) return rc;
  const int tr = trace_begin(st, SS_TRACE_FILTER);
  switch (st->L.W) {
    case 1: launch_filter_w<1>(st, f, ep); break;
    case 2: launch_filter_w<2>(st, f, ep); break;
    default: launch_filter_w<4>(st, f, ep); break;
  }
  trace_end(st, tr, entry_bytes(st->L.W), 1, ep, entry_bytes(st->L.W));
  rc = check_launch(st);
  if (rc) return rc;
  after_emit(st, ep, st->n_ub, false, 0);
  return SS_OK;
}

FilterOp base_filter(const ss_state* st, uint32_t inst) {
  FilterOp f{};
  f.has_inst = st->L.has_inst ? 1u : 0u;
  f.iword = st->L.iword;
  f.ishift = st->L.ishift;
  f.imask = st->L.imask;
  f.inst = inst;
  return f;
}

// ---------------------------------------------------------------------------
// op validation and conversion
// ---------------------------------------------------------------------------

int validate_op(const ss_state* st, const ss_op& op) {
  const uint32_t nr = (uint32_t)st->L.regs.size();
  if (op.kind > SS_DIV || op.flags != 0 || op.nctl > 3) return SS_E_ARG;
  if (op.reg >= nr || st->L.regs[op.reg].width == 0) return SS_E_ARG;
  const RegInfo& d = st->L.regs[op.reg];
  for (uint32_t j = 0; j < op.nctl; ++j) {
    const ss_ctl& c = op.ctl[j];
    if (c.reg >= nr || c.qubit >= st->L.regs[c.reg].width || c.value > 1) return SS_E_ARG;
  }
  // a second register (source, address, factor, divisor) must be live too
  auto live = [&](uint64_t r) { return r < nr && st->L.regs[r].width > 0; };
  if ((op.kind == SS_ADD || op.kind == SS_SUB || op.kind == SS_XOR || op.kind == SS_QRAM_LOAD ||
       op.kind == SS_QRAM_UNLOAD || op.kind == SS_MUL || op.kind == SS_DIV) && !live(op.reg2))
    return SS_E_ARG;
  if ((op.kind == SS_MUL || op.kind == SS_DIV) && !live(op.aux)) return SS_E_ARG;
  if (op.kind == SS_DIV && !live(op.imm)) return SS_E_ARG;
  switch (op.kind) {
    case SS_X:
    case SS_H:
    case SS_RY:
    case SS_Y:
    case SS_Z:
    case SS_S:
    case SS_SDG:
    case SS_T:
    case SS_TDG:
    case SS_PHASE:
    case SS_ROT:
      if (op.qmask == 0 || (op.qmask & ~d.mask)) return SS_E_ARG;
      for (uint32_t j = 0; j < op.nctl; ++j)
        if (op.ctl[j].reg == op.reg && ((op.qmask >> op.ctl[j].qubit) & 1ull)) return SS_E_ARG;
      if ((op.kind == SS_RY || op.kind == SS_PHASE) && !std::isfinite(op.theta)) return SS_E_ARG;
      if (op.kind == SS_ROT && (op.aux >= st->mats.size() || __builtin_popcountll(op.qmask) != 1)) return SS_E_ARG;
      return SS_OK;
    case SS_ADDC:
      break;
    case SS_MUL:
      if (op.reg2 >= nr || op.aux >= nr || op.reg2 == op.reg || op.aux == op.reg) return SS_E_ARG;
      break;
    case SS_DIV: {
      // quotient reg, remainder imm; dividend reg2, divisor aux
      if (op.reg2 >= nr || op.aux >= nr || op.imm >= nr) return SS_E_ARG;
      const uint64_t rr = op.imm;
      if (rr == op.reg || op.reg2 == op.reg || op.aux == op.reg || op.reg2 == rr || op.aux == rr) return SS_E_ARG;
      for (uint32_t j = 0; j < op.nctl; ++j)
        if (op.ctl[j].reg == rr) return SS_E_ARG;
      break;
    }
    case SS_ADD:
    case SS_SUB:
    case SS_XOR:
      if (op.reg2 >= nr || op.reg2 == op.reg) return SS_E_ARG;
      break;
    case SS_MULC:
      if ((op.imm & 1ull) == 0) return SS_E_NOT_UNITARY;
      break;
    case SS_XORC:
    case SS_REFLECT0:
      break;
    case SS_QRAM_LOAD:
    case SS_QRAM_UNLOAD: {
      if (op.reg2 >= nr || op.reg2 == op.reg) return SS_E_ARG;
      if (op.aux >= st->tables.size()) return SS_E_QRAM;
      const TableInfo& t = st->tables[op.aux];
      if (st->L.regs[op.reg2].width != t.addr_bits || d.width != t.word_bits) return SS_E_QRAM;
      break;
    }
  }
  if (op.kind != SS_REFLECT0)
    for (uint32_t j = 0; j < op.nctl; ++j)
      if (op.ctl[j].reg == op.reg) return SS_E_ARG;
  return SS_OK;
}

void ctl_masks(const ss_state* st, const ss_op& op, uint64_t* cmask, uint64_t* cval) {
  for (int w = 0; w < kMaxW; ++w) cmask[w] = cval[w] = 0;
  for (uint32_t j = 0; j < op.nctl; ++j) {
    const RegInfo& r = st->L.regs[op.ctl[j].reg];
    const uint64_t bit = 1ull << (r.shift + op.ctl[j].qubit);
    cmask[r.word] |= bit;
    if (op.ctl[j].value) cval[r.word] |= bit;
  }
}

PermOp to_perm(const ss_state* st, const ss_op& op) {
  PermOp p{};
  const RegInfo& d = st->L.regs[op.reg];
  p.dst_word = d.word;
  p.dst_shift = d.shift;
  p.dst_mask = d.mask;
  p.src_word = 0;
  p.src_shift = 0;
  p.src_mask = 0;
  switch (op.kind) {
    case SS_X: p.kind = PK_XMASK; p.imm = op.qmask & d.mask; break;
    case SS_XORC: p.kind = PK_XORC; p.imm = op.imm & d.mask; break;
    case SS_MULC: p.kind = PK_MULC; p.imm = op.imm; break;
    case SS_ADD: p.kind = PK_ADD; break;
    case SS_SUB: p.kind = PK_SUB; break;
    case SS_XOR: p.kind = PK_XOR; break;
    case SS_QRAM_LOAD:
    case SS_QRAM_UNLOAD: {
      p.kind = PK_QRAM;
      const TableInfo& t = st->tables[op.aux];
      p.table = t.dev;
      p.table_words32 = t.w32 ? 1u : 0u;
      break;
    }
    case SS_REFLECT0: p.kind = PK_REFLECT0; break;
    case SS_ADDC: p.kind = PK_ADDC; p.imm = op.imm & d.mask; break;
    case SS_MUL:
    case SS_DIV: {
      p.kind = op.kind == SS_MUL ? PK_MUL : PK_DIV;
      const RegInfo& y = st->L.regs[op.aux];
      p.src2_word = y.word;
      p.src2_shift = y.shift;
      p.src2_mask = y.mask;
      if (op.kind == SS_DIV) {
        const RegInfo& r = st->L.regs[op.imm];
        p.dst2_word = r.word;
        p.dst2_shift = r.shift;
        p.dst2_mask = r.mask;
      }
      break;
    }
    default: {
      bool flip;
      if (one_to_one(st, op, &flip, p.fac)) {
        p.kind = flip ? PK_ADIAG : PK_DIAG;
        p.imm = (op.qmask & d.mask) << d.shift;
      }
      break;
    }
  }
  if (op.kind == SS_ADD || op.kind == SS_SUB || op.kind == SS_XOR || op.kind == SS_QRAM_LOAD ||
      op.kind == SS_QRAM_UNLOAD || op.kind == SS_MUL || op.kind == SS_DIV) {
    const RegInfo& s = st->L.regs[op.reg2];
    p.src_word = s.word;
    p.src_shift = s.shift;
    p.src_mask = s.mask;
  }
  ctl_masks(st, op, p.cmask, p.cval);
  p.nctl_words = op.nctl ? 1u : 0u;
  return p;
}

// Does a non-branching op keep every group of the mask g contiguous and intact?
bool keeps_grouping(const ss_state* st, const ss_op& op, const uint64_t* g) {
  bool flip;
  double fac[2][2];
  const bool oto = one_to_one(st, op, &flip, fac);
  if (op.kind == SS_REFLECT0 || (oto && !flip)) return true;  // phase only, keys unchanged
  uint64_t reads[kMaxW] = {0, 0, 0, 0}, writes[kMaxW] = {0, 0, 0, 0};
  uint64_t cm[kMaxW], cv[kMaxW];
  ctl_masks(st, op, cm, cv);
  for (int w = 0; w < kMaxW; ++w) reads[w] |= cm[w];
  const RegInfo& d = st->L.regs[op.reg];
  writes[d.word] |= d.mask << d.shift;
  if (op.kind == SS_ADD || op.kind == SS_SUB || op.kind == SS_XOR || op.kind == SS_QRAM_LOAD ||
      op.kind == SS_QRAM_UNLOAD || op.kind == SS_MUL || op.kind == SS_DIV) {
    const RegInfo& s = st->L.regs[op.reg2];
    reads[s.word] |= s.mask << s.shift;
  }
  if (op.kind == SS_MUL || op.kind == SS_DIV) {
    const RegInfo& s = st->L.regs[op.aux];
    reads[s.word] |= s.mask << s.shift;
  }
  if (op.kind == SS_DIV) {
    const RegInfo& r = st->L.regs[op.imm];
    writes[r.word] |= r.mask << r.shift;
  }
  // an xor by a value that does not depend on the group's bits keeps each
  // group's members together (a one-to-one op with a flip xors its mask)
  const bool xor_like = op.kind == SS_X || op.kind == SS_XORC || op.kind == SS_XOR ||
                        op.kind == SS_QRAM_LOAD || op.kind == SS_QRAM_UNLOAD || op.kind == SS_MUL ||
                        op.kind == SS_DIV || oto;
  for (int w = 0; w < kMaxW; ++w) {
    if (reads[w] & g[w]) return false;
    if (!xor_like && (writes[w] & g[w])) return false;
  }
  return true;
}

// Position of a key bit range inside the 32-bit halves of the key words.
struct HalfField {
  bool ok;            // the range lies inside one half
  uint32_t half, sh;  // half index (word*2 + upper) and shift within it
  uint32_t mask;      // width mask (unshifted)
};

HalfField half_of(const RegInfo& r) {
  HalfField f{};
  const uint32_t lo = r.shift % 32;
  f.ok = r.width <= 32 && lo + r.width <= 32;
  f.half = r.word * 2 + (r.shift >= 32 ? 1u : 0u);
  f.sh = lo;
  f.mask = r.width >= 32 ? 0xFFFFFFFFu : ((1u << r.width) - 1u);
  return f;
}

// 32-bit encoding of a non-branching op, or F_GEN when it has no such form.
FastOp encode_fast(const ss_state* st, const ss_op& op, uint32_t gi) {
  FastOp f{};
  f.code = F_GEN;
  f.e = gi;
  const RegInfo& d = st->L.regs[op.reg];
  const HalfField hd = half_of(d);
  auto ctl_bit = [&](const ss_ctl& c, uint32_t& half, uint32_t& bit) {
    const RegInfo& r = st->L.regs[c.reg];
    const uint32_t b = r.shift + c.qubit;
    half = r.word * 2 + (b >= 32 ? 1u : 0u);
    bit = b % 32;
  };
  switch (op.kind) {
    case SS_X:
    case SS_XORC: {
      const uint64_t m64 = ((op.kind == SS_X ? op.qmask : op.imm) & d.mask) << d.shift;
      uint32_t half, imm;
      if ((m64 >> 32) == 0) {
        half = d.word * 2;
        imm = (uint32_t)m64;
      } else if ((m64 & 0xFFFFFFFFull) == 0) {
        half = d.word * 2 + 1;
        imm = (uint32_t)(m64 >> 32);
      } else {
        return f;
      }
      f.imm = imm;
      if (op.nctl == 0) {
        f.code = F_XM + half;
      } else if (op.nctl == 1) {
        uint32_t hc, cb;
        ctl_bit(op.ctl[0], hc, cb);
        f.a = cb;
        f.code = (op.ctl[0].value ? F_XC1 : F_XC1N) + half * 4 + hc;
      } else if (op.nctl == 2) {
        uint32_t hc, cb, hc2, cb2;
        ctl_bit(op.ctl[0], hc, cb);
        ctl_bit(op.ctl[1], hc2, cb2);
        f.a = cb;
        f.b = cb2;
        f.c = op.ctl[0].value ? 0u : ~0u;
        f.d = op.ctl[1].value ? 0u : ~0u;
        f.code = F_XC2 + half * 16 + hc * 4 + hc2;
      }
      return f;
    }
    default:
      break;
  }
  if (op.nctl != 0 || !hd.ok) return f;
  f.a = hd.sh;
  f.b = hd.mask << hd.sh;
  const bool dwhole = hd.mask == 0xFFFFFFFFu;
  switch (op.kind) {
    case SS_ADD:
    case SS_SUB:
    case SS_XOR: {
      const HalfField hs = half_of(st->L.regs[op.reg2]);
      if (!hs.ok) return f;
      f.c = hs.sh;
      // only the low min(widths) source bits reach a result taken modulo
      // 2^(destination width); in a field form that count is below 32
      f.d = std::min<uint32_t>(st->L.regs[op.reg2].width, d.width);
      const bool whole = dwhole && hs.mask == 0xFFFFFFFFu;
      const uint32_t idx = hd.half * 4 + hs.half;
      if (op.kind == SS_ADD) f.code = (whole ? F_ADDA : F_ADDF) + idx;
      else if (op.kind == SS_SUB) f.code = (whole ? F_SUBA : F_SUBF) + idx;
      else f.code = (whole ? F_XORA : F_XORF) + idx;
      return f;
    }
    case SS_MULC:
      f.imm = (uint32_t)op.imm;
      f.d = d.width;
      f.code = (dwhole ? F_MULA : F_MULF) + hd.half;
      return f;
    case SS_QRAM_LOAD:
    case SS_QRAM_UNLOAD: {
      const TableInfo& t = st->tables[op.aux];
      const HalfField hs = half_of(st->L.regs[op.reg2]);
      if (!t.w32 || !hs.ok) return f;
      f.c = hs.sh;
      f.d = hs.mask;
      f.e = (uint32_t)reinterpret_cast<uintptr_t>(t.dev);
      f.f = (uint32_t)(reinterpret_cast<uintptr_t>(t.dev) >> 32);
      f.code = F_QRAM + hd.half * 4 + hs.half;
      return f;
    }
    case SS_REFLECT0:
      f.code = F_REFL + hd.half;
      return f;
    default:
      return f;
  }
}

template <int W>
void launch_perm_w(ss_state* st, const void* dev, uint32_t nfast, const PermOp* gops, uint32_t write_words,
                   bool amp, uint32_t ep) {
  launch_perm<W>(ctx(st), st->perm_entries, amp, static_cast<const FastOp*>(dev), nfast, gops, write_words, ep);
}

// Copy `bytes` into the pinned staging ring and on to the device op ring (on
// the stream); *dev gets the device address.  A full ring waits for the
// stream (a synchronisation) before reuse.
int ring_upload(ss_state* st, const void* src, uint64_t bytes, char** dev) {
  const uint64_t need = align_up(std::max<uint64_t>(bytes, 1), kAlign);
  if (need > kOpRingBytes) return SS_E_ARG;
  if (st->ops_used + need > kOpRingBytes) {
    const int rc = sync_state(st);
    if (rc) return rc;
    if (st->ops_used + need > kOpRingBytes) return SS_E_ARG;
  }
  char* h = reinterpret_cast<char*>(st->hops) + st->ops_used;
  char* d = reinterpret_cast<char*>(st->dev_ops) + st->ops_used;
  if (st->gmode == ss_state::G_CAPTURE) {
    // a graph copies from records it owns (the staging ring is reused)
    if (st->cap_used + need > st->cap_size) return hip_fail(st);
    h = st->cap_hops + st->cap_used;
    st->cap_used += need;
  } else if (st->gmode == ss_state::G_RECORD) {
    st->rec_bytes += need;
  }
  if (bytes) {
    std::memcpy(h, src, bytes);
    if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st->stream) != hipSuccess) return hip_fail(st);
  }
  st->ops_used += need;
  *dev = d;
  return SS_OK;
}

// One fused launch of non-branching ops: its op range, and once uploaded the
// device address of its records (FastOps for W <= 2, then generic records).
struct RunChunk {
  uint64_t first;
  uint32_t len;
  uint32_t write_words;
  bool amp;
  uint64_t fbytes;
  char* dev;
};

// Op ranges of the launches of a call: the runs of non-branching ops, at
// most kRunChunk ops per launch.
void plan_runs(const ss_state* st, const ss_op* ops, uint64_t nops, std::vector<RunChunk>& chunks) {
  uint64_t i = 0;
  while (i < nops) {
    if (is_branching(st, ops[i])) {
      ++i;
      continue;
    }
    uint64_t j = i;
    while (j < nops && !is_branching(st, ops[j]) && j - i < kRunChunk) ++j;
    RunChunk c{};
    c.first = i;
    c.len = (uint32_t)(j - i);
    chunks.push_back(c);
    i = j;
  }
}

// Encode chunks [a, b) into one blob and upload it with one copy.  Encoding
// depends on the register layout only.
int upload_chunks(ss_state* st, const ss_op* ops, std::vector<RunChunk>& chunks, size_t a, size_t b) {
  const uint32_t W = st->L.W;
  std::vector<char> blob;
  std::vector<uint64_t> off(b - a);
  for (size_t k = a; k < b; ++k) {
    RunChunk& c = chunks[k];
    std::vector<FastOp> fast;
    std::vector<PermOp> gen;
    c.write_words = 0;
    c.amp = false;
    for (uint64_t q = c.first; q < c.first + c.len; ++q) {
      const ss_op& op = ops[q];
      if (op_uses_amp(st, op)) c.amp = true;
      c.write_words |= op_write_words(st, op);
      if (W <= 2) {
        FastOp f = encode_fast(st, op, (uint32_t)gen.size());
        if (f.code == F_GEN) gen.push_back(to_perm(st, op));
        fast.push_back(f);
      } else {
        gen.push_back(to_perm(st, op));
      }
    }
    // the interpreter's last prefetch reads one (zero) record past the run
    c.fbytes = fast.empty() ? 0 : align_up((fast.size() + 1) * sizeof(FastOp), kAlign);
    const uint64_t bytes = c.fbytes + gen.size() * sizeof(PermOp);
    off[k - a] = blob.size();
    blob.resize(off[k - a] + align_up(std::max<uint64_t>(bytes, 1), kAlign));
    if (!fast.empty()) std::memcpy(blob.data() + off[k - a], fast.data(), fast.size() * sizeof(FastOp));
    if (!gen.empty()) std::memcpy(blob.data() + off[k - a] + c.fbytes, gen.data(), gen.size() * sizeof(PermOp));
  }
  char* d = nullptr;
  const int rc = ring_upload(st, blob.data(), blob.size(), &d);
  if (rc) return rc;
  for (size_t k = a; k < b; ++k) chunks[k].dev = d + off[k - a];
  return SS_OK;
}

// Launch one uploaded chunk.
int launch_chunk(ss_state* st, const RunChunk& c) {
  const uint32_t W = st->L.W;
  uint32_t ep;
  int rc = begin_launch(st, &ep);
  if (rc) return rc;
  const int tr = trace_begin(st, SS_TRACE_PERM);
  const PermOp* gops = reinterpret_cast<const PermOp*>(c.dev + c.fbytes);
  switch (W) {
    case 1: launch_perm_w<1>(st, c.dev, c.len, gops, c.write_words, c.amp, ep); break;
    case 2: launch_perm_w<2>(st, c.dev, c.len, gops, c.write_words, c.amp, ep); break;
    default: launch_perm_w<4>(st, c.dev, c.len, gops, c.write_words, c.amp, ep); break;
  }
  trace_end(st, tr, 8ull * W + 8ull * (uint64_t)__builtin_popcount(c.write_words) + (c.amp ? 32ull : 0ull), c.len,
            0, 0);
  rc = check_launch(st);
  if (rc) return rc;
  st->masks_valid = false;
  st->mask_ep = ep;
  st->stats[5]++;
  return SS_OK;
}

// One branching op: chunks of at most kMaxGroupBits target qubits, ascending.
// The real 2x2 matrix of a branching op, m[out][in] (host libm).
void gate_matrix(const ss_op& op, double (&m)[2][2]) {
  if (op.kind == SS_ROT) return;  // complex: rot_matrix
  if (op.kind == SS_H) {
    const double c = 0.70710678118654752440;  // nearest double to 1/sqrt(2)
    m[0][0] = c; m[0][1] = c; m[1][0] = c; m[1][1] = -c;
  } else {
    const double h = op.theta / 2.0;
    const double c = std::cos(h), s = std::sin(h);
    m[0][0] = c; m[0][1] = -s; m[1][0] = s; m[1][1] = c;
  }
}

// Ops that can follow `a` in one chained launch: branching on the same one
// target qubit (H or Ry, any controls; controls never include the target).
bool chains_with(const ss_op& a, const ss_op& b) {
  return (b.kind == SS_H || b.kind == SS_RY) && (a.kind == SS_H || a.kind == SS_RY) && b.reg == a.reg &&
         b.qmask == a.qmask && __builtin_popcountll(a.qmask) == 1;
}

// Longest chain for a state's eps.  A chained launch prunes once, after its
// last op, where the plain method prunes after every op.  A prune removes from
// each group amplitudes below eps, a change of norm below sqrt(2)*eps, and the
// later matrices are unitary, so each prune left out moves the result by less
// than that.  The chain is cut so that the sum stays within 1e-12 (the
// amplitude tolerance of the method's results); with eps = 0 the prunes only
// remove exact zeros, which change nothing later.
uint64_t max_chain(double eps) {
  if (!(eps > 0.0)) return (uint64_t)kMaxChain;
  const double k = std::floor(1e-12 / (std::sqrt(2.0) * eps)) + 1.0;
  return k >= (double)kMaxChain ? (uint64_t)kMaxChain : (uint64_t)k;
}

// One branching op, or (nchain >= 2) the one-target ops chain_ops[0..nchain)
// on the same target applied in one launch: each group gets the product of
// the matrices whose controls hold for it, and the prune follows the last.
int do_branching(ss_state* st, const ss_op& op, uint64_t op_index, const ss_op* chain_ops = nullptr,
                 uint32_t nchain = 0, const FusedRun& run = FusedRun{nullptr, 0u, nullptr}) {
  set_mark(st, op_index);
  const RegInfo& d = st->L.regs[op.reg];
  std::vector<uint32_t> qs;
  for (uint32_t q = 0; q < d.width; ++q)
    if ((op.qmask >> q) & 1ull) qs.push_back(q);
  double m[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  gate_matrix(op, m);
  const bool cplx = op.kind == SS_ROT;
  Mat2 cm{};
  if (cplx) {
    cm = st->mats[op.aux];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) m[a][b] = cm.re[a][b];
  }
  // An op split over several launches cannot be rolled back once its first
  // part has run, so it is admitted only if the worst case fits.
  if (qs.size() > (size_t)kMaxGroupBits) {
    if (qs.size() >= 40) return SS_E_CAPACITY;
    auto fits = [&](uint64_t n) { return (n << qs.size()) <= st->cap && ((n << qs.size()) >> qs.size()) == n; };
    if (!fits(st->n_ub)) {
      int rc = ensure_n(st);
      if (rc) return rc;
      if (!fits(st->n)) return SS_E_CAPACITY;
    }
  }
  // A pure expansion (no target bit can vary, by the exact masks or by the
  // host superset) takes up to kMaxExpandBits targets per launch, one thread
  // per child; the check above bounds its output by the capacity.
  size_t chunk = kMaxGroupBits;
  if (st->expand_slots && nchain < 2 && qs.size() > (size_t)kMaxGroupBits) {
    uint64_t tm = 0;
    for (uint32_t q : qs) tm |= 1ull << (d.shift + q);
    const uint64_t var = st->masks_valid ? (st->orm[d.word] & ~st->andm[d.word])
                         : st->sup_valid  ? (st->sorm[d.word] & ~st->sandm[d.word])
                                          : ~0ull;
    if ((var & tm) == 0) chunk = kMaxExpandBits;
  }
  for (size_t c0 = 0; c0 < qs.size(); c0 += chunk) {
    if (st->n_ub == 0) return SS_OK;
    const size_t c1 = std::min(qs.size(), c0 + chunk);
    const bool last = c1 == qs.size();
    GroupOp g{};
    g.k = (uint32_t)(c1 - c0);
    g.upd = c0 == 0 ? 1u : 0u;
    std::vector<std::pair<uint32_t, uint32_t>> tl;
    for (size_t j = c0; j < c1; ++j) {
      const uint32_t bit = d.shift + qs[j];
      g.tword[j - c0] = d.word;
      g.tbit[j - c0] = bit;
      g.tmask[d.word] |= 1ull << bit;
      tl.push_back({d.word, bit});
    }
    ctl_masks(st, op, g.cmask, g.cval);
    g.has_ctl = op.nctl ? 1u : 0u;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g.m[a][b] = m[a][b];
        g.mi[a][b] = cplx ? cm.im[a][b] : 0.0;
      }
    g.cplx = cplx ? 1u : 0u;
    g.eps2 = last ? st->eps * st->eps : 0.0;
    if (nchain >= 2) {
      std::vector<ChainStep> steps(nchain);
      for (uint32_t q = 0; q < nchain; ++q) {
        gate_matrix(chain_ops[q], steps[q].m);
        ctl_masks(st, chain_ops[q], steps[q].cmask, steps[q].cval);
      }
      char* dchain = nullptr;
      int rc = ring_upload(st, steps.data(), steps.size() * sizeof(ChainStep), &dchain);
      if (rc) return rc;
      g.nchain = nchain;
      g.chain = reinterpret_cast<const ChainStep*>(dchain);
      g.upd = nchain;
    }

    int mode;
    bool same = st->grouped && st->grouping;
    for (int w = 0; w < kMaxW && same; ++w) same = st->gmask[w] == g.tmask[w];
    bool sup_const = !st->masks_valid && st->sup_valid;
    for (int w = 0; w < kMaxW && sup_const; ++w) sup_const = ((st->sorm[w] & ~st->sandm[w]) & g.tmask[w]) == 0;
    if (same) {
      mode = MODE_GROUP;
    } else if (sup_const) {
      // no target bit can vary: every group has one member
      mode = MODE_EXPAND;
    } else if (!st->masks_valid && st->sup_valid && st->n_ub <= kSmallSort) {
      // a small state sorts on the bits that may vary rather than wait for
      // the exact masks (an extra radix pass costs less than a read-back);
      // group mode also handles the groups that have one member
      uint64_t var[kMaxW];
      for (int w = 0; w < kMaxW; ++w) var[w] = st->sorm[w] & ~st->sandm[w];
      SortPlan plan;
      build_plan(st->L.W, tl, g.tmask, var, plan);
      int rc = run_sort(st, plan);
      if (rc) return rc;
      mode = MODE_GROUP;
    } else {
      int rc = ensure_masks(st);
      if (rc) return rc;
      bool tvar = false;
      uint64_t var[kMaxW];
      for (int w = 0; w < kMaxW; ++w) {
        var[w] = st->orm[w] & ~st->andm[w];
        if (var[w] & g.tmask[w]) tvar = true;
      }
      if (!tvar) {
        mode = MODE_EXPAND;
      } else {
        SortPlan plan;
        build_plan(st->L.W, tl, g.tmask, var, plan);
        rc = run_sort(st, plan);
        if (rc) return rc;
        mode = MODE_GROUP;
      }
      if (st->n_ub == 0) return SS_OK;
    }
    // more than kMaxGroupBits targets only as a pure expansion
    if (g.k > (uint32_t)kMaxGroupBits && mode != MODE_EXPAND) return SS_E_STATE;
    // one-target op on many entries: try the fixed placement first (two
    // children per entry in expand mode, one in group mode; no look-back);
    // the compacting launch after it finishes the op either way.
    uint32_t ep_spec = 0, ep;
    int rc = SS_OK;
    if (g.k == 1 && ((mode == MODE_EXPAND && st->speculate && st->n_est >= st->speculate) ||
                     (mode == MODE_GROUP && st->spec_group && st->n_est >= st->spec_group))) {
      if (st->spec_skip[mode]) {
        --st->spec_skip[mode];
      } else {
        rc = begin_launch(st, &ep_spec);
        ++st->spec_tries[mode];
      }
    }
    if (!rc) rc = begin_launch(st, &ep);
    if (rc) return rc;
    const uint32_t cat = mode == MODE_GROUP ? SS_TRACE_GROUP : SS_TRACE_EXPAND;
    const int tr = trace_begin(st, cat);
    switch (st->L.W) {
      case 1: launch_group_w<1>(st, mode, g, ep, ep_spec, run); break;
      case 2: launch_group_w<2>(st, mode, g, ep, ep_spec, run); break;
      default: launch_group_w<4>(st, mode, g, ep, ep_spec, FusedRun{nullptr, 0u, nullptr}); break;
    }
    trace_end(st, tr, entry_bytes(st->L.W), 1, ep, entry_bytes(st->L.W));
    rc = check_launch(st);
    if (rc) return rc;
    st->stats[mode == MODE_GROUP ? 3 : 4]++;
    const uint64_t est = mode == MODE_EXPAND ? st->n_est << g.k : st->n_est;
    after_emit(st, ep, st->n_ub << g.k, true, op_index);
    st->n_est = std::min(est, st->n_ub);
    for (int w = 0; w < kMaxW; ++w) sup_vary(st, (uint32_t)w, g.tmask[w]);
    st->grouped = true;
    for (int w = 0; w < kMaxW; ++w) st->gmask[w] = g.tmask[w];
  }
  return SS_OK;
}

int check_state(const ss_state* st) {
  if (!st) return SS_E_STATE;
  if (st->poisoned) return SS_E_STATE;
  return SS_OK;
}

int setup_arena(ss_state* st, char* arena, size_t bytes) {
  const uint32_t W = st->L.W;
  // largest capacity (multiple of 256) whose carve fits
  uint64_t lo = 0, hi = bytes / (2 * entry_bytes(W)) + 1;
  while (lo + 1 < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (carve(W, st->ninst, mid * 256, st->table_bytes).total <= bytes) lo = mid;
    else hi = mid;
  }
  const uint64_t cap = lo * 256;
  if (cap < std::max<uint64_t>(256, st->ninst)) return SS_E_NOMEM;
  st->cap = cap;
  st->cv = carve(W, st->ninst, cap, st->table_bytes);
  st->arena = arena;
  st->arena_bytes = bytes;
  st->meta = reinterpret_cast<DevMeta*>(arena + st->cv.meta);
  st->digit_start = reinterpret_cast<uint64_t*>(arena + st->cv.digit_start);
  st->dev_ops = reinterpret_cast<PermOp*>(arena + st->cv.dev_ops);
  st->uscr = reinterpret_cast<uint64_t*>(arena + st->cv.uscr);
  st->hist = reinterpret_cast<unsigned long long*>(arena + st->cv.hist);
  st->tab_base = arena + st->cv.tables;
  st->lb = reinterpret_cast<uint64_t*>(arena + st->cv.lb);
  st->buf[0] = make_buf(arena + st->cv.buf0, W, cap);
  st->buf[1] = make_buf(arena + st->cv.buf1, W, cap);
  return SS_OK;
}

int init_device(ss_state* st) {
  k_meta_init<<<1, 64, 0, st->stream>>>(st->meta);
  k_fill_u64<<<256, 256, 0, st->stream>>>(st->lb, st->cv.lb_words, 0ull);
  // Which XCD runs each of 64 workgroups: per-XCD tile tickets are used only
  // when equal residues of blockIdx % 8 share an XCD and residues differ by XCD.
  k_xcc_probe<<<64, 64, 0, st->stream>>>(st->uscr);
  st->stats[0] += 3;
  int rc = check_launch(st);
  if (rc) return rc;
  uint64_t ids[64];
  if (hipMemcpyAsync(ids, st->uscr, sizeof(ids), hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipStreamSynchronize(st->stream) != hipSuccess)
    return hip_fail(st);
  // residue classes of blockIdx % 8 map one-to-one onto XCDs
  bool rr = true;
  for (int i = 0; i < 64; ++i) rr = rr && ids[i] == ids[i % kXcds];
  for (int i = 0; i < kXcds; ++i)
    for (int j = 0; j < i; ++j) rr = rr && ids[i] != ids[j];
  st->xcd_order = rr ? 1u : 0u;
  // histogram grids: a multiple of the workgroups resident on the device
  // (occupancy x CUs)
  for (int i = 0; i < 3; ++i) {
    const uint32_t r = sort_hist_resident(i == 0 ? 1u : i == 1 ? 2u : 4u);
    if (r == 0) return hip_fail(st);
    st->hist_res[i] = kHistWaves * r;
  }
  // device meta is fresh: empty state in slot 0, no pending launches
  st->epoch = 0;
  st->nslot = 0;
  set_known(st, 0);
  st->masks_valid = false;
  st->mask_ep = 0;
  st->grouped = false;
  st->emits.clear();
  st->ops_used = 0;
  return SS_OK;
}

template <int W>
void launch_pack(ss_state* st, const uint64_t* values, const double2* amps, uint64_t n, uint64_t at,
                 const PackDesc& pd) {
  const Buf& b = st->buf[st->cur];
  k_pack<W><<<(uint32_t)((n + 255) / 256), 256, 0, st->stream>>>(values, amps, n, kp<W>(b), b.amp, at, pd);
}

// Append n entries (register values, row-major, and amplitudes; host arrays)
// at the current exact count, staged through the alternate buffer; the
// instance field gets `inst`, or `inst` + row index with `row_inst`.
// Whether the n entries given as register values (row-major n x nregs,
// truncated to the register widths) have distinct keys: the packed keys are
// sorted on the host and neighbours compared.
bool keys_distinct(const ss_state* st, const uint64_t* values, uint64_t n) {
  const uint32_t nr = (uint32_t)st->L.regs.size(), W = st->L.W;
  std::vector<uint64_t> k(n * W, 0);
  for (uint64_t i = 0; i < n; ++i)
    for (uint32_t r = 0; r < nr; ++r) {
      const RegInfo& ri = st->L.regs[r];
      k[i * W + ri.word] |= (values[i * nr + r] & ri.mask) << ri.shift;
    }
  std::vector<uint64_t> idx(n);
  for (uint64_t i = 0; i < n; ++i) idx[i] = i;
  auto less = [&](uint64_t a, uint64_t b) {
    for (int w = (int)W - 1; w >= 0; --w)
      if (k[a * W + w] != k[b * W + w]) return k[a * W + w] < k[b * W + w];
    return false;
  };
  std::sort(idx.begin(), idx.end(), less);
  for (uint64_t i = 1; i < n; ++i)
    if (!less(idx[i - 1], idx[i])) return false;
  return true;
}

int pack_entries(ss_state* st, const uint64_t* values, const double* amps, uint64_t n, uint32_t inst,
                 bool row_inst) {
  const uint32_t nr = (uint32_t)st->L.regs.size();
  PackDesc pd{};
  pd.nregs = nr;
  pd.has_inst = st->L.has_inst ? (row_inst ? 2u : 1u) : 0u;
  pd.iword = st->L.iword;
  pd.ishift = st->L.ishift;
  pd.inst = inst;
  for (uint32_t r = 0; r < nr; ++r) {
    pd.word[r] = st->L.regs[r].word;
    pd.shift[r] = st->L.regs[r].shift;
    pd.mask[r] = st->L.regs[r].mask;
  }
  // superset masks: the imported keys' exact OR / AND, joined with those of
  // the entries kept
  {
    uint64_t o[kMaxW] = {0, 0, 0, 0}, a[kMaxW] = {~0ull, ~0ull, ~0ull, ~0ull};
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t k[kMaxW] = {0, 0, 0, 0};
      for (uint32_t r = 0; r < nr; ++r) k[pd.word[r]] |= (values[i * nr + r] & pd.mask[r]) << pd.shift[r];
      if (pd.has_inst) k[pd.iword] |= (pd.has_inst == 2 ? inst + i : (uint64_t)inst) << pd.ishift;
      for (int w = 0; w < kMaxW; ++w) {
        o[w] |= k[w];
        a[w] &= k[w];
      }
    }
    if (st->n == 0) {
      for (int w = 0; w < kMaxW; ++w) {
        st->sorm[w] = o[w];
        st->sandm[w] = a[w];
      }
      st->sup_valid = true;
    } else if (st->sup_valid) {
      for (int w = 0; w < kMaxW; ++w) {
        st->sorm[w] |= o[w];
        st->sandm[w] &= a[w];
      }
    }
  }
  const Buf& alt = st->buf[st->cur ^ 1];
  char* stage = reinterpret_cast<char*>(alt.key[0]);
  const uint64_t stage_bytes = st->cap * entry_bytes(st->L.W);
  const uint64_t per = (uint64_t)nr * 8 + 16;
  const uint64_t chunk = std::max<uint64_t>(1, stage_bytes / per - 1);
  uint64_t done = 0;
  while (done < n) {
    const uint64_t c = std::min(chunk, n - done);
    uint64_t* dv = reinterpret_cast<uint64_t*>(stage);
    double2* da = reinterpret_cast<double2*>(stage + align_up(c * nr * 8, 16));
    if (hipMemcpyAsync(dv, values + done * nr, c * nr * 8, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
        hipMemcpyAsync(da, amps + 2 * done, c * 16, hipMemcpyHostToDevice, st->stream) != hipSuccess)
      return hip_fail(st);
    PackDesc pc = pd;
    pc.inst = inst + (row_inst ? done : 0);
    switch (st->L.W) {
      case 1: launch_pack<1>(st, dv, da, c, st->n + done, pc); break;
      case 2: launch_pack<2>(st, dv, da, c, st->n + done, pc); break;
      default: launch_pack<4>(st, dv, da, c, st->n + done, pc); break;
    }
    int rc = check_launch(st);
    if (rc) return rc;
    // the caller's arrays and the staging area are reused by the next chunk
    if (hipStreamSynchronize(st->stream) != hipSuccess) return hip_fail(st);
    st->stats[6]++;
    done += c;
  }
  set_known(st, st->n + n);
  k_set_n<<<1, 64, 0, st->stream>>>(st->meta, st->nslot, st->n);
  st->masks_valid = false;
  st->mask_ep = 0;
  st->grouped = false;
  return check_launch(st);
}

// ---------------------------------------------------------------------------
// Batched rounds (per-instance op lists)
// ---------------------------------------------------------------------------
constexpr int kBatchItems = 4;           // entries per thread in the batched expand / reduce kernels
constexpr uint64_t kBatchGridCap = 4096; // workgroups of the batched perm launch (it strides)
template <int W>
void launch_perm_batched_w(ss_state* st, const FastOp* f, const PermOp* g, const RunRange* runs, uint32_t ww,
                           bool amp, uint32_t ep) {
  const Buf& b = st->buf[st->cur];
  // the bound can be many times the count (it is the last expansion's count
  // after a reduction), so the grid is capped and the kernel strides
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((st->n_ub + kBlock - 1) / kBlock,
                                                                         kBatchGridCap));
  if (amp)
    k_perm_batched<W, true><<<grid, kBlock, 0, st->stream>>>(kp<W>(b), b.amp, st->nslot, f, g, runs, st->L.iword,
                                                             st->L.ishift, st->L.imask, ww, st->meta, ep);
  else
    k_perm_batched<W, false><<<grid, kBlock, 0, st->stream>>>(kp<W>(b), b.amp, st->nslot, f, g, runs, st->L.iword,
                                                              st->L.ishift, st->L.imask, ww, st->meta, ep);
}

template <int W>
void launch_expand_batched_w(ss_state* st, const BatchOp* bops, uint32_t ep) {
  const Buf& in = st->buf[st->cur];
  const Buf& out = st->buf[st->cur ^ 1];
  constexpr uint64_t T = (uint64_t)kBlock * kBatchItems;
  const uint32_t ntiles = ticket_grid((st->n_ub + T - 1) / T, xo(st));
  k_expand_batched<W, kBatchItems><<<ntiles, kBlock, 0, st->stream>>>(kp<W>(in), in.amp, kp<W>(out), out.amp, st->nslot,
                                                         st->cap, bops, st->L.iword, st->L.ishift, st->L.imask,
                                                         st->lb, st->meta, ep, xo(st));
}

template <int W>
void launch_reduce_batched_w(ss_state* st, const BatchOp* bops, uint32_t ep) {
  const Buf& in = st->buf[st->cur];
  const Buf& out = st->buf[st->cur ^ 1];
  constexpr uint64_t T = (uint64_t)kBlock * kBatchItems;
  const uint32_t ntiles = ticket_grid((st->n_ub + T - 1) / T, xo(st));
  k_reduce_batched<W, kBatchItems><<<ntiles, kBlock, 0, st->stream>>>(kp<W>(in), in.amp, kp<W>(out), out.amp, st->nslot,
                                                         st->cap, bops, st->L.iword, st->L.ishift, st->L.imask,
                                                         st->lb, st->meta, ep, xo(st));
}

template <int W>
void launch_relabel_w(ss_state* st, const uint32_t* map, bool reset, uint32_t gen, uint32_t ep) {
  const Buf& b = st->buf[st->cur];
  const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, (st->n_ub + kBlock - 1) / kBlock), 4096);
  k_relabel<W><<<grid, kBlock, 0, st->stream>>>(kp<W>(b), st->nslot, st->L.iword, st->L.ishift, st->L.imask, map,
                                                 reset ? 1u : 0u, gen, st->meta, ep);
}

template <int W>
void launch_retire_w(ss_state* st, uint32_t a, uint32_t gen, uint32_t ep) {
  const Buf& in = st->buf[st->cur];
  const Buf& out = st->buf[st->cur ^ 1];
  constexpr uint64_t T = (uint64_t)kBlock * 4;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, (st->n_ub + T - 1) / T), 2048);
  k_retire_copy<W><<<grid, kBlock, 0, st->stream>>>(kp<W>(in), in.amp, kp<W>(out), out.amp, st->nslot, st->L.iword,
                                                     st->L.ishift, st->L.imask, a, st->meta, ep);
  k_retire_set<<<1, 64, 0, st->stream>>>(st->meta, gen, 0u);
}

// Relabel the instance field of every entry through `map` (label -> value);
// with `reset` the batched view ends (base = 0).  No map: only the reset.
int relabel_entries(ss_state* st, const std::vector<uint32_t>& map, bool reset) {
  const uint32_t gen = reset ? ++st->vgen : st->vgen;
  if (map.empty()) {
    if (!reset) return SS_OK;
    k_retire_set<<<1, 64, 0, st->stream>>>(st->meta, gen, 1u);
    return check_launch(st);
  }
  char* d = nullptr;
  int rc = ring_upload(st, map.data(), map.size() * sizeof(uint32_t), &d);
  if (rc) return rc;
  uint32_t ep;
  rc = begin_launch(st, &ep);
  if (rc) return rc;
  const uint32_t* m = reinterpret_cast<const uint32_t*>(d);
  switch (st->L.W) {
    case 1: launch_relabel_w<1>(st, m, reset, gen, ep); break;
    case 2: launch_relabel_w<2>(st, m, reset, gen, ep); break;
    default: launch_relabel_w<4>(st, m, reset, gen, ep); break;
  }
  rc = check_launch(st);
  if (rc) return rc;
  st->masks_valid = false;
  st->mask_ep = ep;
  st->sup_valid = false;
  st->grouped = false;
  return SS_OK;
}

// For each instance, the pass of the batched loop below in which it runs its
// last op (the loop's control depends on the op lists only).
std::vector<uint64_t> batched_finish_passes(const ss_state* st, const ss_op* ops, const uint64_t* off) {
  const uint32_t NI = st->ninst;
  std::vector<uint64_t> cur(off, off + NI), end(off + 1, off + NI + 1), fin(NI, 0);
  std::vector<uint32_t> chunk(NI, 0);
  uint64_t pass = 0;
  while (true) {
    ++pass;
    bool any_run = false, any_branch = false;
    for (uint32_t i = 0; i < NI; ++i) {
      if (chunk[i] != 0) continue;
      uint64_t j = cur[i];
      while (j < end[i] && !is_branching(st, ops[j])) ++j;
      any_run = any_run || j > cur[i];
      cur[i] = j;
    }
    for (uint32_t i = 0; i < NI; ++i) {
      if (cur[i] >= end[i]) continue;
      const ss_op& op = ops[cur[i]];
      const uint32_t nq = (uint32_t)__builtin_popcountll(op.qmask & st->L.regs[op.reg].mask);
      if ((uint64_t)(chunk[i] + 1) * kMaxGroupBits >= nq) {
        chunk[i] = 0;
        cur[i]++;
      } else {
        chunk[i]++;
      }
      any_branch = true;
    }
    for (uint32_t i = 0; i < NI; ++i)
      if (fin[i] == 0 && cur[i] >= end[i] && chunk[i] == 0) fin[i] = pass;
    if (!any_branch && !any_run) break;
    bool left = false;
    for (uint32_t i = 0; i < NI; ++i) left = left || cur[i] < end[i];
    if (!left) break;
  }
  for (uint32_t i = 0; i < NI; ++i)
    if (fin[i] == 0) fin[i] = pass;
  return fin;
}

int batched_rounds(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* off, ss_result* res,
                   const std::vector<uint32_t>& label, const std::vector<uint64_t>& fin);

// Every instance i runs ops[off[i] .. off[i+1]).  Round r: one fused launch
// advances each instance through its non-branching ops up to its next
// branching op; then one expansion applies each instance's branching op (up to
// five target qubits; wider ops take several rounds), one LSD sort orders the
// candidates by (instance, key) and one reduce-by-key merges equal keys.
// Instances are first relabelled so that labels ascend with the pass of their
// last op; after each round the finished ones (a prefix of the sorted
// entries) are retired, so later rounds move only the entries of unfinished
// instances; at the end the labels go back.
int apply_batched(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* off, ss_result* res) {
  const uint32_t NI = st->ninst;
  if (off[0] != 0 || off[NI] > nops) return SS_E_ARG;
  for (uint32_t i = 0; i < NI; ++i)
    if (off[i] > off[i + 1]) return SS_E_ARG;
  std::vector<uint32_t> label(NI);
  std::vector<uint64_t> fin;
  for (uint32_t i = 0; i < NI; ++i) label[i] = i;
  const bool retire = st->retire_batched && NI > 1 && st->L.has_inst;
  st->undo_map.clear();
  if (retire) {
    fin = batched_finish_passes(st, ops, off);
    std::vector<uint32_t> order(NI);
    for (uint32_t i = 0; i < NI; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return fin[x] < fin[y]; });
    bool ident = true;
    for (uint32_t r = 0; r < NI; ++r) {
      label[order[r]] = r;
      ident = ident && order[r] == r;
    }
    if (!ident) {
      if (st->n_ub > 0) {
        const int rc = relabel_entries(st, label, false);
        if (rc) return rc;
      }
      st->undo_map = order;
    }
  }
  st->in_view = retire;
  const int rc = batched_rounds(st, ops, nops, off, res, label, fin);
  st->in_view = false;
  if (retire && !st->poisoned &&
      (rc == SS_OK || ((rc == SS_E_CAPACITY || rc == SS_E_PLAN) && st->rolled_back))) {
    // labels back to instances, base back to 0 (also after a roll-back: the
    // round input it returned to is still relabelled)
    const int uc = relabel_entries(st, st->undo_map, true);
    if (uc) return uc;
  }
  return rc;
}

int batched_rounds(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* off, ss_result* res,
                   const std::vector<uint32_t>& label, const std::vector<uint64_t>& fin) {
  const uint32_t NI = st->ninst;
  (void)res;
  const bool retire = !fin.empty();
  uint64_t pass = 0;
  uint32_t retired = 0;           // labels below this are retired
  std::vector<uint64_t> fin_l(retire ? NI : 0);
  if (retire)
    for (uint32_t i = 0; i < NI; ++i) fin_l[label[i]] = fin[i];
  std::vector<uint64_t> cur(off, off + NI), end(off + 1, off + NI + 1);
  std::vector<uint32_t> chunk(NI, 0);
  const uint32_t W = st->L.W;
  uint64_t round = 0;
  std::vector<RunRange> runs(NI);
  std::vector<BatchOp> bops(NI);
  // a replay's check can return only to a round's input (after its runs)
  set_mark(st, 0, false);
  st->sup_valid = false;
  while (true) {
    ++pass;
    // --- non-branching runs -------------------------------------------------
    bool any_run = false;
    uint32_t i0 = 0;
    while (i0 < NI) {
      std::vector<FastOp> fast;
      std::vector<PermOp> gen;
      uint32_t ww = 0;
      bool amp = false;
      std::fill(runs.begin(), runs.end(), RunRange{0u, 0u});
      uint32_t i = i0;
      for (; i < NI; ++i) {
        if (chunk[i] != 0) continue;
        uint64_t j = cur[i];
        uint64_t len = 0;
        while (j + len < end[i] && !is_branching(st, ops[j + len])) ++len;
        if (len == 0) continue;
        // keep one launch's op tables well inside the staging ring
        const uint64_t bytes = (fast.size() + len) * sizeof(FastOp) + (gen.size() + len) * sizeof(PermOp);
        if (!fast.empty() && bytes > kOpRingBytes / 2) break;
        runs[label[i]].start = (uint32_t)fast.size();
        runs[label[i]].len = (uint32_t)len;
        for (uint64_t q = 0; q < len; ++q) {
          const ss_op& op = ops[j + q];
          if (op_uses_amp(st, op)) amp = true;
          ww |= op_write_words(st, op);
          FastOp f = W <= 2 ? encode_fast(st, op, (uint32_t)gen.size()) : FastOp{};
          if (W > 2) {
            f.code = F_GEN;
            f.e = (uint32_t)gen.size();
          }
          if (f.code == F_GEN) gen.push_back(to_perm(st, op));
          fast.push_back(f);
        }
        cur[i] = j + len;
      }
      if (!fast.empty() && st->n_ub > 0) {
        // one upload: run table, fast ops, generic ops (a full ring
        // synchronises, which must not happen between parts of one launch)
        const uint64_t o_f = align_up(NI * sizeof(RunRange), kAlign);
        const uint64_t o_g = o_f + align_up(fast.size() * sizeof(FastOp), kAlign);
        std::vector<char> blob(o_g + gen.size() * sizeof(PermOp));
        std::memcpy(blob.data(), runs.data(), NI * sizeof(RunRange));
        std::memcpy(blob.data() + o_f, fast.data(), fast.size() * sizeof(FastOp));
        if (!gen.empty()) std::memcpy(blob.data() + o_g, gen.data(), gen.size() * sizeof(PermOp));
        char* d = nullptr;
        int rc = ring_upload(st, blob.data(), blob.size(), &d);
        if (rc) return rc;
        uint32_t ep;
        rc = begin_launch(st, &ep);
        if (rc) return rc;
        const int tr = trace_begin(st, SS_TRACE_PERM);
        const FastOp* f = reinterpret_cast<const FastOp*>(d + o_f);
        const PermOp* g = reinterpret_cast<const PermOp*>(d + o_g);
        const RunRange* r = reinterpret_cast<const RunRange*>(d);
        if (W == 1) launch_perm_batched_w<1>(st, f, g, r, ww, amp, ep);
        else if (W == 2) launch_perm_batched_w<2>(st, f, g, r, ww, amp, ep);
        else launch_perm_batched_w<4>(st, f, g, r, ww, amp, ep);
        trace_end(st, tr, 8ull * W + 8ull * (uint64_t)__builtin_popcount(ww) + (amp ? 32ull : 0ull), 1, 0, 0);
        rc = check_launch(st);
        if (rc) return rc;
        st->masks_valid = false;
        st->mask_ep = ep;
        st->stats[5]++;
        any_run = true;
      }
      i0 = i;
    }
    // --- branching ops --------------------------------------------------------
    bool any_branch = false;
    for (uint32_t i = 0; i < NI; ++i) {
      BatchOp& b = bops[label[i]];
      b = BatchOp{};
      if (cur[i] >= end[i]) continue;
      const ss_op& op = ops[cur[i]];
      const RegInfo& d = st->L.regs[op.reg];
      std::vector<uint32_t> qs;
      for (uint32_t q = 0; q < d.width; ++q)
        if ((op.qmask >> q) & 1ull) qs.push_back(q);
      const size_t c0 = (size_t)chunk[i] * kMaxGroupBits, c1 = std::min(qs.size(), c0 + kMaxGroupBits);
      const bool last = c1 == qs.size();
      b.k = (uint32_t)(c1 - c0);
      for (size_t j = c0; j < c1; ++j) {
        b.tword[j - c0] = d.word;
        b.tbit[j - c0] = d.shift + qs[j];
      }
      ctl_masks(st, op, b.cmask, b.cval);
      b.has_ctl = op.nctl ? 1u : 0u;
      if (op.kind == SS_ROT) {
        const Mat2& mm = st->mats[op.aux];
        b.cplx = 1;
        for (int r = 0; r < 2; ++r)
          for (int q = 0; q < 2; ++q) {
            b.m[r][q] = mm.re[r][q];
            b.mi[r][q] = mm.im[r][q];
          }
      } else {
        gate_matrix(op, b.m);
      }
      b.prune = 1;
      b.eps2 = last ? st->eps * st->eps : 0.0;
      if (last) {
        chunk[i] = 0;
        cur[i]++;
      } else {
        chunk[i]++;
      }
      any_branch = true;
    }
    if (!any_branch) {
      if (!any_run) break;
      bool left = false;
      for (uint32_t i = 0; i < NI; ++i) left = left || cur[i] < end[i];
      if (!left) break;
      continue;
    }
    ++round;
    if (st->n_ub == 0) continue;
    uint32_t kmax = 0;
    for (uint32_t i = 0; i < NI; ++i) kmax = std::max(kmax, bops[i].k);
    char* db = nullptr;
    int rc = ring_upload(st, bops.data(), NI * sizeof(BatchOp), &db);
    if (rc) return rc;
    const BatchOp* bo = reinterpret_cast<const BatchOp*>(db);
    // expand (capacity-checked; a failure rolls back to this round's input)
    uint32_t ep;
    rc = begin_launch(st, &ep);
    if (rc) return rc;
    int tr = trace_begin(st, SS_TRACE_EXPAND);
    if (W == 1) launch_expand_batched_w<1>(st, bo, ep);
    else if (W == 2) launch_expand_batched_w<2>(st, bo, ep);
    else launch_expand_batched_w<4>(st, bo, ep);
    trace_end(st, tr, entry_bytes(W), 1, ep, entry_bytes(W));
    rc = check_launch(st);
    if (rc) return rc;
    set_mark(st, round);
    after_emit(st, ep, st->n_ub << kmax, true, round);
    // sort candidates by (instance, key): the plan needs the key masks
    rc = ensure_masks(st);
    if (rc) return rc;
    uint64_t var[kMaxW], skip[kMaxW] = {0, 0, 0, 0};
    for (int w = 0; w < kMaxW; ++w) var[w] = st->orm[w] & ~st->andm[w];
    SortPlan plan;
    build_plan(W, {}, skip, var, plan);
    rc = run_sort(st, plan);
    if (rc) return rc;
    // reduce by key + prune
    rc = begin_launch(st, &ep);
    if (rc) return rc;
    tr = trace_begin(st, SS_TRACE_FILTER);
    if (W == 1) launch_reduce_batched_w<1>(st, bo, ep);
    else if (W == 2) launch_reduce_batched_w<2>(st, bo, ep);
    else launch_reduce_batched_w<4>(st, bo, ep);
    trace_end(st, tr, entry_bytes(W), 1, ep, entry_bytes(W));
    rc = check_launch(st);
    if (rc) return rc;
    after_emit(st, ep, st->n_ub, false, round);
    set_mark(st, round + 1, false);
    // retire the instances whose last op ran in this pass: their labels are
    // the next ones up, their entries the start of the view
    if (retire) {
      uint32_t a = retired;
      while (a < NI && fin_l[a] <= pass) ++a;
      if (a > retired) {
        rc = begin_launch(st, &ep);
        if (rc) return rc;
        const uint32_t gen = ++st->vgen;
        if (W == 1) launch_retire_w<1>(st, a, gen, ep);
        else if (W == 2) launch_retire_w<2>(st, a, gen, ep);
        else launch_retire_w<4>(st, a, gen, ep);
        rc = check_launch(st);
        if (rc) return rc;
        retired = a;
      }
    }
  }
  st->grouped = false;
  return SS_OK;
}

int validate_ops(ss_state* st, const ss_op* ops, uint64_t nops, ss_result* res) {
  if (nops && !ops) return SS_E_ARG;
  for (uint64_t i = 0; i < nops; ++i) {
    const int rc = validate_op(st, ops[i]);
    if (rc) {
      res->status = rc;
      res->failed_op = i;
      return rc;
    }
  }
  return SS_OK;
}

// Plan and launch a validated op list; ends with a synchronisation, whose
// status is the call's.
int plan_ops(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* inst_offsets, ss_result* res) {
  auto finish = [&](int code, uint64_t op) {
    // the status is final only after a synchronisation; a capacity failure
    // found there names the op (batched: round) whose launch was rolled back
    st->ops_keep = 0;           // no launch of this call is still to come
    st->final_sync = true;
    const int sc = st->poisoned ? SS_OK : sync_state(st);
    st->final_sync = false;
    if (sc == SS_E_CAPACITY) {
      code = sc;
      op = st->rb_op;
    } else if (sc != SS_OK) {
      code = sc;
    }
    res->status = code;
    res->failed_op = code ? op : 0;
    res->nnz = st->n;
    res->peak = st->peak;
    return code;
  };
  int rc;
  st->ops_keep = 0;
  if (inst_offsets) {
    rc = apply_batched(st, ops, nops, inst_offsets, res);
    if (rc == SS_E_CAPACITY && st->rolled_back) return finish(rc, st->rb_op);
    return finish(rc, 0);
  }
  set_mark(st, 0);
  std::vector<RunChunk> chunks;
  plan_runs(st, ops, nops, chunks);
  size_t ci = 0, up = 0;
  // Records are encoded and uploaded a group of chunks (>= kUploadOps ops) at
  // a time, when the first of them is needed, so that the host encodes while
  // the device runs earlier launches and one copy serves several runs.
  auto ensure_up = [&](size_t c) -> int {
    if (c < up) return SS_OK;
    size_t b = c;
    uint64_t nops_group = 0, bytes = 0;
    while (b < chunks.size() && (b == c || nops_group < kUploadOps)) {
      const uint64_t cb = (uint64_t)chunks[b].len * (sizeof(FastOp) + sizeof(PermOp)) + 2 * kAlign;
      if (b > c && bytes + cb > kOpRingBytes / 2) break;
      nops_group += chunks[b].len;
      bytes += cb;
      ++b;
    }
    const int r = upload_chunks(st, ops, chunks, c, b);
    if (r) return r;
    up = b;
    st->ops_keep = st->ops_used;
    return SS_OK;
  };
  // launch the chunks of ops before `upto`
  auto flush = [&](uint64_t upto) -> int {
    for (; ci < chunks.size() && chunks[ci].first < upto; ++ci) {
      if (st->n_ub == 0) continue;
      set_mark(st, chunks[ci].first);
      int r = ensure_up(ci);
      if (r) return r;
      r = launch_chunk(st, chunks[ci]);
      if (r) return r;
      if (ci + 1 == up) st->ops_keep = 0;
    }
    return SS_OK;
  };
  for (uint64_t i = 0; i < nops; ++i) {
    const ss_op& op = ops[i];
    if (is_branching(st, op)) {
      uint64_t j = i + 1;
      if (st->chain) {
        const uint64_t lim = max_chain(st->eps);
        while (j < nops && j - i < lim && chains_with(op, ops[j])) ++j;
      }
      rc = flush(i);
      // a one-target op takes the run that follows it into its own launch
      FusedRun fr{nullptr, 0u, nullptr};
      const bool fuse = !rc && st->L.W <= 2 && __builtin_popcountll(op.qmask) == 1 && ci < chunks.size() &&
                        chunks[ci].first == j && chunks[ci].len <= st->fuse_runs && st->n_ub > 0;
      if (fuse) {
        set_mark(st, i);
        rc = ensure_up(ci);
        fr = FusedRun{reinterpret_cast<const FastOp*>(chunks[ci].dev), chunks[ci].len,
                      reinterpret_cast<const PermOp*>(chunks[ci].dev + chunks[ci].fbytes)};
      }
      if (!rc) {
        const uint32_t nch = j - i >= 2 ? (uint32_t)(j - i) : 0u;
        rc = do_branching(st, op, i, nch ? ops + i : nullptr, nch, fr);
      }
      if (!rc && fuse) {
        // the run went with the op
        ++ci;
        if (ci >= up) st->ops_keep = 0;
        st->stats[5]++;
      }
      if (rc) {
        if (rc == SS_E_CAPACITY && st->rolled_back) return finish(rc, st->rb_op);
        return finish(rc, i);
      }
      i = j - 1;
    } else {
      if (st->grouped && !keeps_grouping(st, op, st->gmask)) st->grouped = false;
      sup_op(st, op);
    }
  }
  rc = flush(nops);
  if (rc == SS_E_CAPACITY && st->rolled_back) return finish(rc, st->rb_op);
  set_mark(st, nops);
  return finish(rc, nops);
}

// Host planner state saved around a capture (which must plan from the same
// starting point as the recording run and leave the state as that run did).
struct PlanSnap {
  int cur;
  uint32_t nslot;
  uint64_t n, n_ub, n_est, peak;
  bool n_known, masks_valid, grouped, poisoned, sup_valid;
  uint32_t n_src_ep, mask_ep, epoch, ops_used, dev_err, spec_skip[2], spec_backoff[2], spec_tries[2];
  uint64_t spec_fail_seen[2];
  uint64_t orm[kMaxW], andm[kMaxW], gmask[kMaxW], sorm[kMaxW], sandm[kMaxW];
  uint64_t stats[8];
};

PlanSnap save_plan(const ss_state* st) {
  PlanSnap p{};
  p.cur = st->cur;
  p.nslot = st->nslot;
  p.n = st->n;
  p.n_ub = st->n_ub;
  p.n_est = st->n_est;
  p.peak = st->peak;
  p.n_known = st->n_known;
  p.masks_valid = st->masks_valid;
  p.grouped = st->grouped;
  p.poisoned = st->poisoned;
  p.sup_valid = st->sup_valid;
  p.n_src_ep = st->n_src_ep;
  p.mask_ep = st->mask_ep;
  p.epoch = st->epoch;
  p.ops_used = st->ops_used;
  p.dev_err = st->dev_err;
  for (int md = 0; md < 2; ++md) {
    p.spec_skip[md] = st->spec_skip[md];
    p.spec_backoff[md] = st->spec_backoff[md];
    p.spec_tries[md] = st->spec_tries[md];
    p.spec_fail_seen[md] = st->spec_fail_seen[md];
  }
  for (int w = 0; w < kMaxW; ++w) {
    p.orm[w] = st->orm[w];
    p.andm[w] = st->andm[w];
    p.gmask[w] = st->gmask[w];
    p.sorm[w] = st->sorm[w];
    p.sandm[w] = st->sandm[w];
  }
  for (int i = 0; i < 8; ++i) p.stats[i] = st->stats[i];
  return p;
}

void restore_plan(ss_state* st, const PlanSnap& p) {
  st->cur = p.cur;
  st->nslot = p.nslot;
  st->n = p.n;
  st->n_ub = p.n_ub;
  st->n_est = p.n_est;
  st->peak = p.peak;
  st->n_known = p.n_known;
  st->masks_valid = p.masks_valid;
  st->grouped = p.grouped;
  st->poisoned = p.poisoned;
  st->sup_valid = p.sup_valid;
  st->n_src_ep = p.n_src_ep;
  st->mask_ep = p.mask_ep;
  st->epoch = p.epoch;
  st->ops_used = p.ops_used;
  st->dev_err = p.dev_err;
  for (int md = 0; md < 2; ++md) {
    st->spec_skip[md] = p.spec_skip[md];
    st->spec_backoff[md] = p.spec_backoff[md];
    st->spec_tries[md] = p.spec_tries[md];
    st->spec_fail_seen[md] = p.spec_fail_seen[md];
  }
  for (int w = 0; w < kMaxW; ++w) {
    st->orm[w] = p.orm[w];
    st->andm[w] = p.andm[w];
    st->gmask[w] = p.gmask[w];
    st->sorm[w] = p.sorm[w];
    st->sandm[w] = p.sandm[w];
  }
  for (int i = 0; i < 8; ++i) st->stats[i] = p.stats[i];
}

// Move the entries to the other buffer and count slot (count read on the
// device).  Asynchronous.
template <int W>
void launch_copy_w(ss_state* st) {
  const Buf& in = st->buf[st->cur];
  const Buf& out = st->buf[st->cur ^ 1];
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((st->n_ub + kBlock - 1) / kBlock, 4096));
  k_copy_state<W><<<grid, kBlock, 0, st->stream>>>(kp<W>(in), in.amp, kp<W>(out), out.amp, st->nslot, st->meta);
}

int launch_copy(ss_state* st) {
  switch (st->L.W) {
    case 1: launch_copy_w<1>(st); break;
    case 2: launch_copy_w<2>(st); break;
    default: launch_copy_w<4>(st); break;
  }
  st->cur ^= 1;
  st->nslot ^= 1;
  st->stats[0]++;
  return check_launch(st);
}

}  // namespace

// A captured op list: the instantiated graph, the pinned op records its copy
// nodes read, where its plan starts and ends, and the rollback points of its
// launches and checks.
struct ss_graph {
  ss_state* st = nullptr;
  char* arena = nullptr;
  uint64_t cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* hops = nullptr;
  int cur0 = 0;
  uint32_t nslot0 = 0;
  uint64_t n0 = 0;              // entry count the plan starts from
  uint64_t n_end = 0;           // ... and ends with
  bool grouped_end = false;
  uint64_t gmask_end[kMaxW]{};
  uint32_t epoch_end = 0;
  uint64_t kernels = 0;
  std::vector<ss_state::EmitLog> emits;
  std::vector<ss_state::PlanMark> plan_log;
  bool batched_view = false;      // the plan retires instances (batched rounds)
  std::vector<uint32_t> undo_map; // its relabelling, undone after a failed replay
};

// The device array behind ss_create_state_noalloc's scratch (64 MiB).
constexpr uint64_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// ---------------------------------------------------------------------------
// Scratch of the state made by ss_create_state_noalloc: the meta block, digit
// starts, op ring, instance scratch, histograms and look-back words live in
// this array, one copy per device, held until the process ends.  Host code
// uses the address hipGetSymbolAddress gives for the current device, never the
// array's name.  The host-side read-back block and op staging of that state
// are static host arrays (no pinned allocation).
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 8;

struct ScratchSlot {
  char* dev = nullptr;     // device address of `scratch` on this device (0: not looked up yet)
  bool busy = false;       // a live state uses it
};
ScratchSlot g_scratch[kMaxDevices];
DevMeta g_hmeta[kMaxDevices];
PermOp g_hops[kMaxDevices][kMaxOpsPerCall];
std::mutex g_scratch_mu;

// Carve of a state whose scratch is the device array: the scratch parts in
// [scratch, scratch + kScratchBytes), tables and the two entry buffers in the
// caller's memory.  Returns false when the capacity leaves no room.
bool carve_split(uint32_t W, uint32_t ninst, uint64_t cap, uint64_t table_bytes, uint64_t* scratch_bytes,
                 uint64_t* data_bytes, Carve* c) {
  *c = carve(W, ninst, cap, table_bytes);
  // scratch: meta .. uscr (offsets below c->tables), then histograms and
  // look-back words; data: tables, buffer 0, buffer 1
  const uint64_t head = c->tables;
  const uint64_t hist_bytes = align_up(max_passes(W) * kRadix * 8, kAlign);
  const uint64_t lb_bytes = align_up(c->lb_words * 8, kAlign);
  *scratch_bytes = head + hist_bytes + lb_bytes;
  *data_bytes = align_up(table_bytes, kAlign) + 2 * align_up(cap * entry_bytes(W), kAlign);
  return *scratch_bytes <= kScratchBytes;
}

int setup_split(ss_state* st, char* scr, char* data, size_t data_bytes) {
  const uint32_t W = st->L.W;
  uint64_t lo = 0, hi = data_bytes / (2 * entry_bytes(W)) / 256 + 1;
  uint64_t sb, db;
  Carve c;
  while (lo + 1 < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (carve_split(W, st->ninst, mid * 256, st->table_bytes, &sb, &db, &c) && db <= data_bytes) lo = mid;
    else hi = mid;
  }
  const uint64_t cap = lo * 256;
  if (cap < std::max<uint64_t>(256, st->ninst)) return SS_E_NOMEM;
  carve_split(W, st->ninst, cap, st->table_bytes, &sb, &db, &c);
  st->cap = cap;
  st->cv = c;
  st->arena = data;
  st->arena_bytes = data_bytes;
  st->meta = reinterpret_cast<DevMeta*>(scr + c.meta);
  st->digit_start = reinterpret_cast<uint64_t*>(scr + c.digit_start);
  st->dev_ops = reinterpret_cast<PermOp*>(scr + c.dev_ops);
  st->uscr = reinterpret_cast<uint64_t*>(scr + c.uscr);
  st->hist = reinterpret_cast<unsigned long long*>(scr + c.tables);
  st->lb = reinterpret_cast<uint64_t*>(scr + c.tables + align_up(max_passes(W) * kRadix * 8, kAlign));
  st->tab_base = data;
  const uint64_t b0 = align_up(st->table_bytes, kAlign);
  st->buf[0] = make_buf(data + b0, W, cap);
  st->buf[1] = make_buf(data + b0 + align_up(cap * entry_bytes(W), kAlign), W, cap);
  return SS_OK;
}

void graph_free(ss_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->hops) (void)hipHostFree(g->hops);
  delete g;
}

}  // namespace

extern "C" {

const char* ss_strerror(int code) {
  switch (code) {
    case SS_OK: return "ok";
    case SS_E_ARG: return "invalid argument";
    case SS_E_NOT_UNITARY: return "operation is not unitary (even multiplier)";
    case SS_E_QRAM: return "invalid QRAM table or QRAM operands";
    case SS_E_CAPACITY: return "entry capacity of the arena exceeded";
    case SS_E_NOMEM: return "arena too small";
    case SS_E_HIP: return "HIP runtime or kernel failure";
    case SS_E_STATE: return "state is null or poisoned";
    case SS_E_PLAN: return "state does not fit the captured plan (rolled back)";
    default: return "unknown error";
  }
}

int ss_required_bytes(const ss_reg* regs, uint32_t nregs, uint32_t ninst, uint64_t cap_entries,
                      uint64_t table_bytes, size_t* bytes) {
  if (!bytes) return SS_E_ARG;
  Layout L;
  int rc = make_layout(regs, nregs, ninst, L);
  if (rc) return rc;
  const uint64_t cap = align_up(std::max<uint64_t>(cap_entries, 256), 256);
  *bytes = carve(L.W, ninst, cap, table_bytes).total;
  return SS_OK;
}

int ss_create_state(const ss_reg* regs, uint32_t nregs, uint32_t ninst, double eps, void* arena,
                    size_t arena_bytes, uint64_t table_bytes, void* hip_stream, ss_state** out) {
  if (!out || !arena || ((uintptr_t)arena % kAlign) || !(eps >= 0.0) || !std::isfinite(eps)) return SS_E_ARG;
  *out = nullptr;
  ss_state* st = new ss_state();
  int rc = make_layout(regs, nregs, ninst, st->L);
  if (rc) {
    delete st;
    return rc;
  }
  st->ninst = ninst;
  st->eps = eps;
  st->stream = static_cast<hipStream_t>(hip_stream);
  st->table_bytes = align_up(table_bytes, kAlign);
  rc = setup_arena(st, static_cast<char*>(arena), arena_bytes);
  if (rc) {
    delete st;
    return rc;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&st->hmeta), sizeof(DevMeta), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&st->hops), (size_t)kMaxOpsPerCall * sizeof(PermOp),
                    hipHostMallocDefault) != hipSuccess) {
    if (st->hmeta) (void)hipHostFree(st->hmeta);
    delete st;
    return SS_E_HIP;
  }
  rc = init_device(st);
  if (rc) {
    ss_destroy_state(st);
    return rc;
  }
  // every instance starts as |0...0> with amplitude 1
  std::vector<uint64_t> vals((size_t)ninst * nregs, 0ull);
  std::vector<double> amps(2 * (size_t)ninst, 0.0);
  for (uint32_t i = 0; i < ninst; ++i) amps[2 * i] = 1.0;
  rc = pack_entries(st, vals.data(), amps.data(), ninst, 0, true);
  if (!rc) rc = sync_state(st);
  if (rc) {
    ss_destroy_state(st);
    return rc;
  }
  *out = st;
  return SS_OK;
}

int ss_create_state_noalloc(const ss_reg* regs, uint32_t nregs, uint32_t ninst, double eps, void* entries,
                            size_t entry_bytes, uint64_t table_bytes, void* hip_stream, ss_state** out) {
  if (!out || !entries || ((uintptr_t)entries % kAlign) || !(eps >= 0.0) || !std::isfinite(eps)) return SS_E_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SS_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return SS_E_ARG;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot& slot = g_scratch[dev];
    if (!slot.dev) {
      // once per device, with that device current
      if (hipGetSymbolAddress(reinterpret_cast<void**>(&slot.dev), HIP_SYMBOL(scratch)) != hipSuccess || !slot.dev) {
        slot.dev = nullptr;
        return SS_E_HIP;
      }
    }
    if (slot.busy) return SS_E_STATE;
    slot.busy = true;
  }
  auto release = [&]() {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch[dev].busy = false;
  };
  ss_state* st = new ss_state();
  st->static_scratch = true;
  st->static_dev = dev;
  int rc = make_layout(regs, nregs, ninst, st->L);
  if (rc) {
    delete st;
    release();
    return rc;
  }
  st->ninst = ninst;
  st->eps = eps;
  st->stream = static_cast<hipStream_t>(hip_stream);
  st->table_bytes = align_up(table_bytes, kAlign);
  rc = setup_split(st, g_scratch[dev].dev, static_cast<char*>(entries), entry_bytes);
  if (rc) {
    delete st;
    release();
    return rc;
  }
  st->hmeta = &g_hmeta[dev];
  st->hops = g_hops[dev];
  rc = init_device(st);
  if (rc) {
    ss_destroy_state(st);
    return rc;
  }
  std::vector<uint64_t> vals((size_t)ninst * nregs, 0ull);
  std::vector<double> amps(2 * (size_t)ninst, 0.0);
  for (uint32_t i = 0; i < ninst; ++i) amps[2 * i] = 1.0;
  rc = pack_entries(st, vals.data(), amps.data(), ninst, 0, true);
  if (!rc) rc = sync_state(st);
  if (rc) {
    ss_destroy_state(st);
    return rc;
  }
  *out = st;
  return SS_OK;
}

int ss_destroy_state(ss_state* st) {
  if (!st) return SS_E_STATE;
  for (ss_graph* g : st->graphs) g->st = nullptr;
  (void)hipStreamSynchronize(st->stream);
  drop_trace(st);
  for (hipEvent_t e : st->ev_pool) (void)hipEventDestroy(e);
  if (st->static_scratch) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch[st->static_dev].busy = false;
  } else {
    if (st->hmeta) (void)hipHostFree(st->hmeta);
    if (st->hops) (void)hipHostFree(st->hops);
  }
  delete st;
  return SS_OK;
}

int ss_capacity(const ss_state* st, uint64_t* cap) {
  if (!st || !cap) return SS_E_ARG;
  *cap = st->cap;
  return SS_OK;
}

int ss_layout(const ss_state* st, uint32_t reg, uint32_t* word, uint32_t* offset, uint32_t* width) {
  if (!st || reg >= st->L.regs.size()) return SS_E_ARG;
  if (word) *word = st->L.regs[reg].word;
  if (offset) *offset = st->L.regs[reg].shift;
  if (width) *width = st->L.regs[reg].width;
  return SS_OK;
}

int ss_key_words(const ss_state* st, uint32_t* w) {
  if (!st || !w) return SS_E_ARG;
  *w = st->L.W;
  return SS_OK;
}

int ss_load_qram(ss_state* st, const uint64_t* table, uint64_t len, uint32_t addr_bits, uint32_t word_bits,
                 uint32_t* qram_id) {
  int rc = check_state(st);
  if (rc) return rc;
  if (!table || !qram_id || addr_bits > 40 || word_bits < 1 || word_bits > 64) return SS_E_QRAM;
  if (len != (1ull << addr_bits)) return SS_E_QRAM;
  const bool w32 = word_bits <= 32;
  std::vector<uint32_t> t32;
  for (uint64_t i = 0; i < len; ++i)
    if (word_bits < 64 && (table[i] >> word_bits)) return SS_E_QRAM;
  const uint64_t bytes = align_up(len * (w32 ? 4 : 8), kAlign);
  if (st->tab_used + bytes > st->table_bytes) return SS_E_NOMEM;
  void* dev = st->tab_base + st->tab_used;
  if (w32) {
    t32.resize(len);
    for (uint64_t i = 0; i < len; ++i) t32[i] = (uint32_t)table[i];
    if (hipMemcpyAsync(dev, t32.data(), len * 4, hipMemcpyHostToDevice, st->stream) != hipSuccess)
      return hip_fail(st);
  } else {
    if (hipMemcpyAsync(dev, table, len * 8, hipMemcpyHostToDevice, st->stream) != hipSuccess)
      return hip_fail(st);
  }
  if (hipStreamSynchronize(st->stream) != hipSuccess) return hip_fail(st);
  st->tab_used += bytes;
  st->tables.push_back({dev, addr_bits, word_bits, w32});
  *qram_id = (uint32_t)st->tables.size() - 1;
  return SS_OK;
}

int ss_load_matrix(ss_state* st, const double* m, uint32_t* matrix_id) {
  int rc = check_state(st);
  if (rc) return rc;
  if (!m || !matrix_id) return SS_E_ARG;
  Mat2 M{};
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      M.re[r][c] = m[4 * r + 2 * c];
      M.im[r][c] = m[4 * r + 2 * c + 1];
      if (!std::isfinite(M.re[r][c]) || !std::isfinite(M.im[r][c])) return SS_E_ARG;
    }
  // unitary: (M^H M)[i][j] = sum_r conj(M[r][i]) M[r][j] within 1e-12 of I
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double re = 0.0, im = 0.0;
      for (int r = 0; r < 2; ++r) {
        re += M.re[r][i] * M.re[r][j] + M.im[r][i] * M.im[r][j];
        im += M.re[r][i] * M.im[r][j] - M.im[r][i] * M.re[r][j];
      }
      if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-12 || std::fabs(im) > 1e-12) return SS_E_NOT_UNITARY;
    }
  st->mats.push_back(M);
  *matrix_id = (uint32_t)st->mats.size() - 1;
  return SS_OK;
}

int ss_set_entries(ss_state* st, uint32_t inst, const uint64_t* values, const double* amps, uint64_t n) {
  int rc = check_state(st);
  if (rc) return rc;
  if (inst >= st->ninst || (n && (!values || !amps))) return SS_E_ARG;
  if (!keys_distinct(st, values, n)) return SS_E_ARG;
  // drop the instance's current entries
  if (st->L.has_inst) {
    FilterOp f = base_filter(st, inst);
    f.kind = FILTER_DROP_INST;
    rc = run_filter(st, f);
    if (!rc) rc = sync_state(st);
    if (rc) return rc;
  } else {
    // every call ends synchronised; wait only if something is still pending
    if (!st->n_known || !st->emits.empty() || !st->plan_log.empty() || !st->pending.empty()) {
      rc = sync_state(st);
      if (rc) return rc;
    }
    set_known(st, 0);
  }
  if (st->n + n > st->cap) {
    k_set_n<<<1, 64, 0, st->stream>>>(st->meta, st->nslot, st->n);
    st->masks_valid = false;
    st->mask_ep = 0;
    st->grouped = false;
    (void)check_launch(st);
    return SS_E_CAPACITY;
  }
  // (pack_entries waits for its copies: the caller's arrays are free on return)
  return pack_entries(st, values, amps, n, inst, false);
}

int ss_apply_ops(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* inst_offsets, ss_result* res) {
  int rc = check_state(st);
  if (rc) return rc;
  ss_result local{};
  if (!res) res = &local;
  *res = ss_result{};
  rc = validate_ops(st, ops, nops, res);
  if (rc) return rc;
  return plan_ops(st, ops, nops, inst_offsets, res);
}

int ss_prune(ss_state* st, double eps) {
  int rc = check_state(st);
  if (rc) return rc;
  if (!(eps >= 0.0)) return SS_E_ARG;
  FilterOp f = base_filter(st, 0);
  f.has_inst = 0;
  f.kind = FILTER_PRUNE;
  f.eps2 = eps * eps;
  rc = run_filter(st, f);
  if (rc) return rc;
  return sync_state(st);
}

int ss_nnz(ss_state* st, uint32_t inst, uint64_t* nnz, uint64_t* peak) {
  int rc = check_state(st);
  if (rc) return rc;
  rc = sync_state(st);
  if (rc) return rc;
  if (peak) *peak = st->peak;
  if (!nnz) return SS_OK;
  if (inst == UINT32_MAX || !st->L.has_inst) {
    *nnz = st->n;
    return SS_OK;
  }
  if (inst >= st->ninst) return SS_E_ARG;
  // count by sorting on the instance field and reading two bounds
  uint64_t lo = 0, hi = 0;
  if (st->n) {
    rc = sort_canonical(st);
    if (rc) return rc;
    const uint32_t W = st->L.W;
    k_fill_u64<<<1, 256, 0, st->stream>>>(st->uscr, st->ninst + 1, st->n);
    const uint32_t g = (uint32_t)((st->n + 255) / 256);
    const Buf& b = st->buf[st->cur];
    if (W == 1) k_inst_bounds<1><<<g, 256, 0, st->stream>>>(kp<1>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    else if (W == 2) k_inst_bounds<2><<<g, 256, 0, st->stream>>>(kp<2>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    else k_inst_bounds<4><<<g, 256, 0, st->stream>>>(kp<4>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    rc = check_launch(st);
    if (rc) return rc;
    uint64_t bnd[2];
    if (hipMemcpyAsync(bnd, st->uscr + inst, 16, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
        hipStreamSynchronize(st->stream) != hipSuccess)
      return hip_fail(st);
    lo = bnd[0];
    hi = bnd[1];
    if (lo > hi || hi > st->n) return hip_fail(st);
  }
  *nnz = hi - lo;
  return SS_OK;
}

int ss_export(ss_state* st, uint32_t inst, uint64_t* keys, double* amps, uint64_t cap, uint64_t* n_out) {
  int rc = check_state(st);
  if (rc) return rc;
  if (inst >= st->ninst || !n_out || (cap && (!keys || !amps))) return SS_E_ARG;
  *n_out = 0;
  rc = sync_state(st);
  if (rc) return rc;
  if (st->n == 0) return SS_OK;
  rc = sort_canonical(st);
  if (rc) return rc;
  const uint32_t W = st->L.W;
  uint64_t lo = 0, hi = st->n;
  const Buf& b = st->buf[st->cur];
  if (st->L.has_inst) {
    k_fill_u64<<<1, 256, 0, st->stream>>>(st->uscr, st->ninst + 1, st->n);
    const uint32_t g = (uint32_t)((st->n + 255) / 256);
    if (W == 1) k_inst_bounds<1><<<g, 256, 0, st->stream>>>(kp<1>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    else if (W == 2) k_inst_bounds<2><<<g, 256, 0, st->stream>>>(kp<2>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    else k_inst_bounds<4><<<g, 256, 0, st->stream>>>(kp<4>(b), st->n, st->L.iword, st->L.ishift, st->L.imask, st->uscr, st->ninst);
    rc = check_launch(st);
    if (rc) return rc;
    uint64_t bnd[2];
    if (hipMemcpyAsync(bnd, st->uscr + inst, 16, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
        hipStreamSynchronize(st->stream) != hipSuccess)
      return hip_fail(st);
    lo = bnd[0];
    hi = bnd[1];
    if (lo > hi || hi > st->n) return hip_fail(st);
  }
  const uint64_t cnt = hi - lo;
  *n_out = cnt;
  const uint64_t m = std::min(cnt, cap);
  if (m == 0) return SS_OK;
  const Buf& alt = st->buf[st->cur ^ 1];
  uint64_t* ok = alt.key[0];
  double2* oa = alt.amp;
  const uint64_t iclear = st->L.has_inst ? (st->L.imask << st->L.ishift) : 0ull;
  const uint32_t iword = st->L.has_inst ? st->L.iword : 99u;
  const uint32_t g = (uint32_t)((m + 255) / 256);
  if (W == 1) k_export<1><<<g, 256, 0, st->stream>>>(kp<1>(b), b.amp, lo, lo + m, ok, oa, iword, iclear);
  else if (W == 2) k_export<2><<<g, 256, 0, st->stream>>>(kp<2>(b), b.amp, lo, lo + m, ok, oa, iword, iclear);
  else k_export<4><<<g, 256, 0, st->stream>>>(kp<4>(b), b.amp, lo, lo + m, ok, oa, iword, iclear);
  rc = check_launch(st);
  if (rc) return rc;
  if (hipMemcpyAsync(keys, ok, m * W * 8, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipMemcpyAsync(amps, oa, m * 16, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipStreamSynchronize(st->stream) != hipSuccess)
    return hip_fail(st);
  return SS_OK;
}

}  // extern "C"

namespace {

// Sort the entries by (instance, field of register reg), so that a running
// sum visits the field's values in ascending order within each instance.
int sort_by_field(ss_state* st, uint32_t reg) {
  int rc = ensure_masks(st);
  if (rc) return rc;
  const RegInfo& r = st->L.regs[reg];
  uint64_t var[kMaxW] = {0, 0, 0, 0}, skip[kMaxW] = {0, 0, 0, 0};
  var[r.word] |= (r.mask << r.shift) & (st->orm[r.word] & ~st->andm[r.word]);
  std::vector<std::pair<uint32_t, uint32_t>> low;
  for (uint32_t b = 0; b < 64; ++b)
    if ((var[r.word] >> b) & 1ull) low.push_back({r.word, b});
  uint64_t ivar[kMaxW] = {0, 0, 0, 0};
  if (st->L.has_inst) ivar[st->L.iword] = (st->L.imask << st->L.ishift) & (st->orm[st->L.iword] & ~st->andm[st->L.iword]);
  SortPlan plan;
  build_plan(st->L.W, low, skip, ivar, plan);
  rc = run_sort(st, plan);
  if (rc) return rc;
  st->grouped = false;
  return SS_OK;
}

template <int W>
void launch_runs_w(ss_state* st, uint64_t n, const FilterOp& f, double* part, uint32_t* fhead, double* tail,
                   double* carry, const double* total, uint64_t* out_val) {
  const Buf& b = st->buf[st->cur];
  const uint32_t ntiles = (uint32_t)((n + kBlock - 1) / kBlock);
  k_runs_tile<W><<<ntiles, kBlock, 0, st->stream>>>(kp<W>(b), b.amp, n, f, part, fhead, tail);
  k_runs_carry<<<1, 64, 0, st->stream>>>(fhead, tail, ntiles, carry);
  k_runs_out<W><<<ntiles, kBlock, 0, st->stream>>>(kp<W>(b), n, f, part, fhead, carry, total, out_val);
}

}  // namespace

extern "C" {

int ss_measure(ss_state* st, uint32_t inst, uint32_t reg, double u, uint64_t* outcome, double* prob) {
  int rc = check_state(st);
  if (rc) return rc;
  if (inst >= st->ninst || reg >= st->L.regs.size() || st->L.regs[reg].width == 0 || !(u >= 0.0 && u < 1.0) ||
      !outcome || !prob)
    return SS_E_ARG;
  rc = sync_state(st);
  if (rc) return rc;
  if (st->n == 0) return SS_E_ARG;
  rc = sort_by_field(st, reg);
  if (rc) return rc;
  const RegInfo& r = st->L.regs[reg];
  const uint32_t W = st->L.W;
  FilterOp f = base_filter(st, inst);
  f.fword = r.word;
  f.fshift = r.shift;
  f.fmask = r.mask;
  const Buf& b = st->buf[st->cur];
  const Buf& alt = st->buf[st->cur ^ 1];
  const uint64_t n = st->n;
  const uint32_t ntiles = (uint32_t)((n + kBlock - 1) / kBlock);
  double* tile_sum = reinterpret_cast<double*>(alt.amp);
  double* incl = tile_sum + align_up(ntiles, 64);
  double* dtot = st->meta->dscratch;
  unsigned long long* out = reinterpret_cast<unsigned long long*>(st->uscr);
  auto tiles = [&](const FilterOp& fo) {
    if (W == 1) k_prob_tiles<1><<<ntiles, kBlock, 0, st->stream>>>(kp<1>(b), b.amp, n, fo, tile_sum);
    else if (W == 2) k_prob_tiles<2><<<ntiles, kBlock, 0, st->stream>>>(kp<2>(b), b.amp, n, fo, tile_sum);
    else k_prob_tiles<4><<<ntiles, kBlock, 0, st->stream>>>(kp<4>(b), b.amp, n, fo, tile_sum);
  };
  f.use_f = 0;
  tiles(f);
  k_prob_scan<<<1, 64, 0, st->stream>>>(tile_sum, ntiles, dtot);
  k_fill_u64<<<1, 64, 0, st->stream>>>(st->uscr, 1, ~0ull);
  k_fill_u64<<<1, 64, 0, st->stream>>>(st->uscr + 1, 3, 0ull);
  if (W == 1) k_prob_find<1><<<ntiles, kBlock, 0, st->stream>>>(kp<1>(b), b.amp, n, f, tile_sum, dtot, u, incl, out);
  else if (W == 2) k_prob_find<2><<<ntiles, kBlock, 0, st->stream>>>(kp<2>(b), b.amp, n, f, tile_sum, dtot, u, incl, out);
  else k_prob_find<4><<<ntiles, kBlock, 0, st->stream>>>(kp<4>(b), b.amp, n, f, tile_sum, dtot, u, incl, out);
  if (W == 1) k_prob_pick<1><<<1, 64, 0, st->stream>>>(kp<1>(b), f, out);
  else if (W == 2) k_prob_pick<2><<<1, 64, 0, st->stream>>>(kp<2>(b), f, out);
  else k_prob_pick<4><<<1, 64, 0, st->stream>>>(kp<4>(b), f, out);
  rc = check_launch(st);
  if (rc) return rc;
  unsigned long long hout[4];
  double P = 0.0;
  if (hipMemcpyAsync(hout, out, 32, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipMemcpyAsync(&P, dtot, 8, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipStreamSynchronize(st->stream) != hipSuccess)
    return hip_fail(st);
  if (!(P > 0.0)) return SS_E_ARG;  // the instance holds no entries
  uint64_t v;
  if (hout[0] != ~0ull) {
    v = hout[1];
  } else {
    // no running sum exceeds u*P (u*P at the total by rounding): the
    // largest field value present
    v = hout[2];
  }
  f.use_f = 1;
  f.fval = v;
  tiles(f);
  k_prob_scan<<<1, 64, 0, st->stream>>>(tile_sum, ntiles, dtot + 1);
  double pv = 0.0;
  if (hipMemcpyAsync(&pv, dtot + 1, 8, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipStreamSynchronize(st->stream) != hipSuccess)
    return hip_fail(st);
  FilterOp c = f;
  c.kind = FILTER_COLLAPSE;
  c.scale = std::sqrt(pv);
  rc = run_filter(st, c);
  if (!rc) rc = sync_state(st);
  if (rc) return rc;
  st->grouped = false;
  *outcome = v;
  *prob = pv / P;
  return SS_OK;
}

int ss_probabilities(ss_state* st, uint32_t inst, uint32_t reg, uint64_t* values, double* probs, uint64_t cap,
                     uint64_t* n_out) {
  int rc = check_state(st);
  if (rc) return rc;
  if (inst >= st->ninst || reg >= st->L.regs.size() || st->L.regs[reg].width == 0 || !n_out ||
      (cap && (!values || !probs)))
    return SS_E_ARG;
  rc = sync_state(st);
  if (rc) return rc;
  *n_out = 0;
  if (st->n == 0) return SS_OK;
  rc = sort_by_field(st, reg);
  if (rc) return rc;
  rc = sync_state(st);
  if (rc) return rc;
  const RegInfo& r = st->L.regs[reg];
  const uint32_t W = st->L.W;
  const uint64_t n = st->n;
  FilterOp f = base_filter(st, inst);
  f.fword = r.word;
  f.fshift = r.shift;
  f.fmask = r.mask;
  f.use_f = 0;
  // scratch in the other entry buffer: per-entry sums / results and field
  // values, then per-tile arrays
  const uint64_t ntiles = (n + kBlock - 1) / kBlock;
  char* base = reinterpret_cast<char*>(st->buf[st->cur ^ 1].key[0]);
  double* part = reinterpret_cast<double*>(base);
  uint64_t* out_val = reinterpret_cast<uint64_t*>(base + align_up(n * 8, kAlign));
  double* tile_sum = reinterpret_cast<double*>(base + 2 * align_up(n * 8, kAlign));
  double* tail = tile_sum + align_up(ntiles, 64);
  double* carry = tail + align_up(ntiles, 64);
  uint32_t* fhead = reinterpret_cast<uint32_t*>(carry + align_up(ntiles, 64));
  double* dtot = st->meta->dscratch + 2;
  const Buf& b = st->buf[st->cur];
  // P: the instance's total, tile sums then one scan in tile order
  if (W == 1) k_prob_tiles<1><<<(uint32_t)ntiles, kBlock, 0, st->stream>>>(kp<1>(b), b.amp, n, f, tile_sum);
  else if (W == 2) k_prob_tiles<2><<<(uint32_t)ntiles, kBlock, 0, st->stream>>>(kp<2>(b), b.amp, n, f, tile_sum);
  else k_prob_tiles<4><<<(uint32_t)ntiles, kBlock, 0, st->stream>>>(kp<4>(b), b.amp, n, f, tile_sum);
  k_prob_scan<<<1, 64, 0, st->stream>>>(tile_sum, ntiles, dtot);
  switch (W) {
    case 1: launch_runs_w<1>(st, n, f, part, fhead, tail, carry, dtot, out_val); break;
    case 2: launch_runs_w<2>(st, n, f, part, fhead, tail, carry, dtot, out_val); break;
    default: launch_runs_w<4>(st, n, f, part, fhead, tail, carry, dtot, out_val); break;
  }
  rc = check_launch(st);
  if (rc) return rc;
  std::vector<double> hp(n);
  std::vector<uint64_t> hv(n);
  if (hipMemcpyAsync(hp.data(), part, n * 8, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipMemcpyAsync(hv.data(), out_val, n * 8, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
      hipStreamSynchronize(st->stream) != hipSuccess)
    return hip_fail(st);
  uint64_t k = 0;
  for (uint64_t e = 0; e < n; ++e) {
    if (!(hp[e] >= 0.0)) continue;   // not the end of one of the instance's field runs
    if (k < cap) {
      values[k] = hv[e];
      probs[k] = hp[e];
    }
    ++k;
  }
  *n_out = k;
  return SS_OK;
}

}  // extern "C"

namespace {

// Lowest run of `width` free bits in the lowest key word (registers and the
// instance field hold bits).
bool place_register(const Layout& L, uint32_t width, uint32_t* word, uint32_t* shift) {
  const uint64_t m0 = width >= 64 ? ~0ull : ((1ull << width) - 1);
  for (uint32_t w = 0; w < (uint32_t)kMaxW; ++w) {
    uint64_t used = 0;
    for (const RegInfo& r : L.regs)
      if (r.width && r.word == w) used |= r.mask << r.shift;
    if (L.has_inst && L.iword == w) used |= L.imask << L.ishift;
    for (uint32_t off = 0; off + width <= 64; ++off)
      if ((used & (m0 << off)) == 0) {
        *word = w;
        *shift = off;
        return true;
      }
  }
  return false;
}

template <int WI, int WO>
void relayout(ss_state* st, const Buf& in, const Buf& out, uint64_t n) {
  if (n == 0) return;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + kBlock - 1) / kBlock, 8192);
  k_relayout<WI, WO><<<grid, kBlock, 0, st->stream>>>(kp<WI>(in), in.amp, kp<WO>(out), out.amp, n);
}

void relayout_any(ss_state* st, uint32_t WI, uint32_t WO, const Buf& in, const Buf& out, uint64_t n) {
  if (WI == 1 && WO == 1) relayout<1, 1>(st, in, out, n);
  else if (WI == 1 && WO == 2) relayout<1, 2>(st, in, out, n);
  else if (WI == 1) relayout<1, 4>(st, in, out, n);
  else if (WI == 2 && WO == 2) relayout<2, 2>(st, in, out, n);
  else if (WI == 2) relayout<2, 4>(st, in, out, n);
  else relayout<4, 4>(st, in, out, n);
}

// Re-carve the arena for keys of W2 > W words and move the entries: into
// buffer 0, then to a staging area at the arena's end with the wider keys
// (new words 0), then into the new buffer 0.  The staging area lies after the
// old buffer 0 and after the new one, so no step overwrites what it reads.
int grow_key_words(ss_state* st, uint32_t W2) {
  int rc = sync_state(st);
  if (rc) return rc;
  const uint32_t W = st->L.W;
  const uint64_t n = st->n, peak = st->peak, upd = st->stats[7];
  // the new capacity: largest multiple of 256 whose carve fits the arena
  uint64_t lo = 0, hi = st->arena_bytes / (2 * entry_bytes(W2)) + 1;
  while (lo + 1 < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (carve(W2, st->ninst, mid * 256, st->table_bytes).total <= st->arena_bytes) lo = mid;
    else hi = mid;
  }
  const uint64_t cap2 = lo * 256;
  if (cap2 < std::max<uint64_t>({n, 256, st->ninst})) return SS_E_NOMEM;
  const Carve c2 = carve(W2, st->ninst, cap2, st->table_bytes);
  const uint64_t nal = align_up(std::max<uint64_t>(n, 2), 2);
  const uint64_t stage_off = (st->arena_bytes - nal * entry_bytes(W2)) / kAlign * kAlign;
  if (st->arena_bytes < nal * entry_bytes(W2) + kAlign || stage_off < st->cv.buf0 + st->cap * entry_bytes(W) ||
      stage_off < c2.buf0 + cap2 * entry_bytes(W2))
    return SS_E_NOMEM;
  const Buf stage = make_buf(st->arena + stage_off, W2, nal);
  if (st->cur == 1) relayout_any(st, W, W, st->buf[1], st->buf[0], n);
  relayout_any(st, W, W2, st->buf[0], stage, n);
  rc = check_launch(st);
  if (rc) return rc;
  st->L.W = W2;
  rc = setup_arena(st, st->arena, st->arena_bytes);
  if (rc) return hip_fail(st);  // cannot happen: the carve was checked above
  relayout_any(st, W2, W2, stage, st->buf[0], n);
  st->cur = 0;
  rc = init_device(st);
  if (rc) return rc;
  const uint64_t spec_fail[2] = {st->spec_fail_seen[0], st->spec_fail_seen[1]};
  if (hipMemcpyAsync(&st->meta->peak, &peak, 8, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
      hipMemcpyAsync(&st->meta->upd, &upd, 8, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
      hipMemcpyAsync(st->meta->spec_fail, spec_fail, 16, hipMemcpyHostToDevice, st->stream) != hipSuccess)
    return hip_fail(st);
  set_known(st, n);
  k_set_n<<<1, 64, 0, st->stream>>>(st->meta, st->nslot, n);
  rc = check_launch(st);
  if (rc) return rc;
  return sync_state(st);
}

// Graphs capture a layout; a register change retires them.
void detach_graphs(ss_state* st) {
  for (ss_graph* g : st->graphs) g->st = nullptr;
  st->graphs.clear();
}

}  // namespace

extern "C" {

int ss_add_register(ss_state* st, uint32_t nqubits, const char* name, uint32_t* reg) {
  (void)name;
  int rc = check_state(st);
  if (rc) return rc;
  if (nqubits < 1 || nqubits > 64 || !reg || st->L.regs.size() >= 64) return SS_E_ARG;
  RegInfo ri{};
  if (!place_register(st->L, nqubits, &ri.word, &ri.shift)) return SS_E_NOMEM;
  ri.width = nqubits;
  ri.mask = nqubits == 64 ? ~0ull : ((1ull << nqubits) - 1);
  const uint32_t need = ri.word + 1;
  const uint32_t W2 = need <= 1 ? 1 : (need <= 2 ? 2 : 4);
  if (W2 > st->L.W) {
    if (st->static_scratch) return SS_E_NOMEM;   // its carve is fixed
    rc = grow_key_words(st, W2);
    if (rc) return rc;
  }
  detach_graphs(st);
  st->L.regs.push_back(ri);
  *reg = (uint32_t)st->L.regs.size() - 1;
  return SS_OK;
}

int ss_remove_register(ss_state* st, uint32_t reg) {
  int rc = check_state(st);
  if (rc) return rc;
  if (reg >= st->L.regs.size() || st->L.regs[reg].width == 0) return SS_E_ARG;
  rc = sync_state(st);
  if (rc) return rc;
  const RegInfo r = st->L.regs[reg];
  uint64_t v = 0;
  if (st->n) {
    rc = ensure_masks(st);
    if (rc) return rc;
    const uint64_t f = r.mask << r.shift;
    if ((st->orm[r.word] ^ st->andm[r.word]) & f) return SS_E_ARG;   // more than one value
    v = (st->orm[r.word] >> r.shift) & r.mask;
  }
  detach_graphs(st);
  if (v) {
    // clear the register's bits: xor its one value
    ss_op op{};
    op.kind = SS_XORC;
    op.reg = reg;
    op.imm = v;
    ss_result res{};
    rc = ss_apply_ops(st, &op, 1, nullptr, &res);
    if (rc) return rc;
  }
  st->L.regs[reg].width = 0;
  st->L.regs[reg].mask = 0;
  return SS_OK;
}

int ss_sync(ss_state* st, ss_result* res) {
  if (!st) return SS_E_STATE;
  const int rc = sync_state(st);
  if (res) {
    res->status = rc;
    res->failed_op = (rc == SS_E_CAPACITY || rc == SS_E_PLAN) ? st->rb_op : 0;
    res->nnz = st->n;
    res->peak = st->peak;
  }
  return rc;
}

int ss_rebind_arena(ss_state* st, void* arena, size_t arena_bytes) {
  int rc = check_state(st);
  if (rc) return rc;
  if (st->static_scratch) return SS_E_ARG;
  if (!arena || ((uintptr_t)arena % kAlign)) return SS_E_ARG;
  rc = sync_state(st);
  if (rc) return rc;
  const uint64_t n = st->n, peak = st->peak, upd = st->stats[7];
  const Buf src = st->buf[st->cur];
  char* old_tab = st->tab_base;
  const uint64_t old_used = st->tab_used;
  struct Saved {
    uint64_t cap;
    Carve cv;
    char* arena;
    size_t arena_bytes;
    DevMeta* meta;
    uint64_t* digit_start;
    PermOp* dev_ops;
    uint64_t* uscr;
    unsigned long long* hist;
    char* tab_base;
    uint64_t* lb;
    Buf b0, b1;
  } old{st->cap, st->cv, st->arena, st->arena_bytes, st->meta, st->digit_start, st->dev_ops,
        st->uscr, st->hist, st->tab_base, st->lb, st->buf[0], st->buf[1]};
  rc = setup_arena(st, static_cast<char*>(arena), arena_bytes);
  if (rc || st->cap < n || st->table_bytes < old_used) {
    // keep the old carve
    st->cap = old.cap;
    st->cv = old.cv;
    st->arena = old.arena;
    st->arena_bytes = old.arena_bytes;
    st->meta = old.meta;
    st->digit_start = old.digit_start;
    st->dev_ops = old.dev_ops;
    st->uscr = old.uscr;
    st->hist = old.hist;
    st->tab_base = old.tab_base;
    st->lb = old.lb;
    st->buf[0] = old.b0;
    st->buf[1] = old.b1;
    return rc ? rc : SS_E_NOMEM;
  }
  st->cur = 0;
  const uint32_t W = st->L.W;
  for (uint32_t w = 0; w < W; ++w)
    if (n && hipMemcpyAsync(st->buf[0].key[w], src.key[w], n * 8, hipMemcpyDeviceToDevice, st->stream) != hipSuccess)
      return hip_fail(st);
  if (n && hipMemcpyAsync(st->buf[0].amp, src.amp, n * 16, hipMemcpyDeviceToDevice, st->stream) != hipSuccess)
    return hip_fail(st);
  if (old_used && hipMemcpyAsync(st->tab_base, old_tab, old_used, hipMemcpyDeviceToDevice, st->stream) != hipSuccess)
    return hip_fail(st);
  for (auto& t : st->tables) t.dev = st->tab_base + (static_cast<char*>(t.dev) - old_tab);
  rc = init_device(st);
  if (rc) return rc;
  const uint64_t spec_fail[2] = {st->spec_fail_seen[0], st->spec_fail_seen[1]};
  if (hipMemcpyAsync(&st->meta->peak, &peak, 8, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
      hipMemcpyAsync(&st->meta->upd, &upd, 8, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
      hipMemcpyAsync(st->meta->spec_fail, spec_fail, 16, hipMemcpyHostToDevice, st->stream) != hipSuccess)
    return hip_fail(st);
  set_known(st, n);
  k_set_n<<<1, 64, 0, st->stream>>>(st->meta, st->nslot, n);
  rc = check_launch(st);
  if (rc) return rc;
  return sync_state(st);
}

int ss_graph_capture(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* inst_offsets,
                     ss_result* res, ss_graph** out) {
  if (!out) return SS_E_ARG;
  *out = nullptr;
  int rc = check_state(st);
  if (rc) return rc;
  if (st->gmode != ss_state::G_EAGER) return SS_E_STATE;
  ss_result local{};
  if (!res) res = &local;
  *res = ss_result{};
  rc = validate_ops(st, ops, nops, res);
  if (rc) return rc;
  // A clean start, as every replay's prologue makes it: exact count, nothing
  // pending, fresh look-back words and ring, epoch 1 (the tag of checks made
  // before the first launch), no masks or grouping carried over.
  rc = sync_state(st);
  if (rc) {
    res->status = rc;
    return rc;
  }
  k_fill_u64<<<1024, 256, 0, st->stream>>>(st->lb, st->cv.lb_words, 0ull);
  k_ring_init<<<1, 64, 0, st->stream>>>(st->meta);
  st->stats[0] += 2;
  if (check_launch(st)) return SS_E_HIP;
  st->epoch = 1;
  st->mask_ep = 0;
  st->masks_valid = false;
  st->sup_valid = false;
  st->grouped = false;
  const PlanSnap p0 = save_plan(st);
  const bool trace = st->trace;
  st->trace = false;
  // 1. the real application, recording every read-back
  st->gmode = ss_state::G_RECORD;
  st->snaps.clear();
  st->rec_bytes = 0;
  rc = plan_ops(st, ops, nops, inst_offsets, res);
  st->gmode = ss_state::G_EAGER;
  if (rc) {
    st->trace = trace;
    st->snaps.clear();
    return rc;
  }
  const PlanSnap p1 = save_plan(st);
  // 2. the same plan under stream capture on a private stream (nothing runs)
  ss_graph* g = new ss_graph();
  g->st = st;
  g->arena = st->arena;
  g->cap = st->cap;
  g->cur0 = p0.cur;
  g->nslot0 = p0.nslot;
  g->n0 = p0.n;
  const uint64_t rec = std::max<uint64_t>(st->rec_bytes, kAlign);
  hipStream_t cs = nullptr;
  int crc = SS_OK;
  if (hipHostMalloc(reinterpret_cast<void**>(&g->hops), rec, hipHostMallocDefault) != hipSuccess ||
      hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    crc = SS_E_HIP;
  if (!crc) {
    hipStream_t real = st->stream;
    restore_plan(st, p0);
    st->stream = cs;
    st->gmode = ss_state::G_CAPTURE;
    st->snap_pos = 0;
    st->cap_hops = g->hops;
    st->cap_used = 0;
    st->cap_size = rec;
    st->emits.clear();
    st->plan_log.clear();
    const uint64_t k0 = st->stats[0];
    (void)hipGetLastError();
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      crc = SS_E_HIP;
    } else {
      // prologue: fresh look-back words and ring, then the input check
      k_fill_u64<<<1024, 256, 0, cs>>>(st->lb, st->cv.lb_words, 0ull);
      k_ring_init<<<1, 64, 0, cs>>>(st->meta);
      k_plan_guard<<<1, 64, 0, cs>>>(st->meta, st->nslot, st->n, -1, PlanVar{}, st->epoch);
      st->plan_log.push_back({st->epoch, st->cur, st->nslot, 0, true});
      st->stats[0] += 3;
      ss_result cres{};
      int prc = check_launch(st);
      if (!prc) prc = plan_ops(st, ops, nops, inst_offsets, &cres);
      if (!prc && (st->poisoned || st->snap_pos != st->snaps.size())) prc = SS_E_HIP;
      // end in the buffer it began in, so that replays chain
      if (!prc && (st->cur != g->cur0 || st->nslot != g->nslot0)) prc = launch_copy(st);
      if (!prc) {
        // epilogue: a clean ring for the launches that follow the replay
        k_ring_init<<<1, 64, 0, cs>>>(st->meta);
        st->stats[0]++;
        prc = check_launch(st);
      }
      g->n_end = st->n;
      g->grouped_end = st->grouped;
      for (int w = 0; w < kMaxW; ++w) g->gmask_end[w] = st->gmask[w];
      g->epoch_end = st->epoch;
      g->emits = st->emits;
      g->plan_log = st->plan_log;
      g->kernels = st->stats[0] - k0;
      g->batched_view = inst_offsets && st->retire_batched && st->ninst > 1 && st->L.has_inst;
      g->undo_map = st->undo_map;
      hipGraph_t graph = nullptr;
      if (hipStreamEndCapture(cs, &graph) != hipSuccess && !prc) prc = SS_E_HIP;
      g->graph = graph;
      crc = prc;
    }
    (void)hipGetLastError();
    st->stream = real;
    st->gmode = ss_state::G_EAGER;
    st->cap_hops = nullptr;
    st->cap_used = st->cap_size = 0;
    restore_plan(st, p1);   // the capture ran nothing on the device
    st->emits.clear();
    st->plan_log.clear();
  }
  st->snaps.clear();
  st->trace = trace;
  if (cs) (void)hipStreamDestroy(cs);
  if (!crc && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) crc = SS_E_HIP;
  (void)hipGetLastError();
  if (crc) {
    graph_free(g);
    return crc;
  }
  st->graphs.push_back(g);
  *out = g;
  return SS_OK;
}

int ss_graph_launch(ss_graph* g, ss_result* res) {
  if (!g) return SS_E_ARG;
  ss_result local{};
  if (!res) res = &local;
  *res = ss_result{};
  ss_state* st = g->st;
  int rc = check_state(st);
  if (rc) return rc;
  if (st->gmode != ss_state::G_EAGER) return SS_E_STATE;
  if (st->arena != g->arena || st->cap != g->cap) return SS_E_ARG;
  if (!st->n_known || !st->emits.empty() || !st->plan_log.empty() || !st->pending.empty()) {
    rc = sync_state(st);
    if (rc) {
      res->status = rc;
      return rc;
    }
  }
  res->nnz = st->n;
  res->peak = st->peak;
  if (st->n != g->n0) {
    res->status = SS_E_PLAN;
    return SS_E_PLAN;
  }
  if (st->cur != g->cur0 || st->nslot != g->nslot0) {
    rc = launch_copy(st);
    if (rc) return rc;
  }
  if (hipGraphLaunch(g->exec, st->stream) != hipSuccess) return hip_fail(st);
  st->stats[0] += g->kernels;
  st->emits = g->emits;
  st->plan_log = g->plan_log;
  st->cur = g->cur0;
  st->nslot = g->nslot0;
  st->n_known = false;
  st->n_ub = g->n_end;
  st->n_est = g->n_end;
  st->n_src_ep = 0;
  st->masks_valid = false;
  st->sup_valid = false;
  st->mask_ep = 0;
  st->grouped = g->grouped_end;
  for (int w = 0; w < kMaxW; ++w) st->gmask[w] = g->gmask_end[w];
  st->epoch = std::max(st->epoch, g->epoch_end);
  rc = sync_state(st);
  if ((rc == SS_E_CAPACITY || rc == SS_E_PLAN) && st->rolled_back && g->batched_view && !st->poisoned) {
    // the replay stopped inside its batched rounds, before it gave the labels
    // and the retired prefix back: do that now
    st->undo_map = g->undo_map;
    const int uc = relabel_entries(st, st->undo_map, true);
    if (uc) return uc;
  }
  res->status = rc;
  res->failed_op = (rc == SS_E_CAPACITY || rc == SS_E_PLAN) ? st->rb_op : 0;
  res->nnz = st->n;
  res->peak = st->peak;
  return rc;
}

int ss_graph_destroy(ss_graph* g) {
  if (!g) return SS_E_ARG;
  if (g->st) {
    auto& v = g->st->graphs;
    v.erase(std::remove(v.begin(), v.end(), g), v.end());
  }
  graph_free(g);
  return SS_OK;
}

int ss_set_option(ss_state* st, const char* key, int64_t value) {
  if (!st || !key) return SS_E_ARG;
  const std::string k(key);
  if (k == "sort_items") {
    if (value != 8 && value != 16) return SS_E_ARG;
    st->sort_items = (int)value;
  } else if (k == "tile_order") {
    // 1: per-XCD tickets when the device spreads workgroups round-robin (one
    // stream; radix passes take them in chunks of consecutive tiles); 0: one
    // ticket counter (states driven concurrently on several streams of one
    // GPU must use 0)
    st->tile_order_opt = value ? 1 : 0;
  } else if (k == "perm_entries") {
    if (value != 4 && value != 8 && value != 16) return SS_E_ARG;
    st->perm_entries = (int)value;
  } else if (k == "group_items") {
    if (value != 1 && value != 2 && value != 4) return SS_E_ARG;
    st->group_items = (int)value;
  } else if (k == "grouping") {
    st->grouping = value ? 1 : 0;
  } else if (k == "speculate") {
    if (value < 0) return SS_E_ARG;
    st->speculate = (uint64_t)value;
  } else if (k == "chain") {
    st->chain = value ? 1 : 0;
  } else if (k == "retire") {
    if (value != 0 && value != 1) return SS_E_ARG;
    st->retire_batched = value != 0;
  } else if (k == "fuse_runs") {
    if (value < 0 || value > (int64_t)kRunChunk) return SS_E_ARG;
    st->fuse_runs = (uint32_t)value;
  } else if (k == "pair_exchange") {
    if (value < 0 || value > 2) return SS_E_ARG;
    st->pair_exchange = (uint32_t)value;
  } else if (k == "expand_slots") {
    st->expand_slots = value ? 1 : 0;
  } else if (k == "spec_items") {
    if (value != 1 && value != 2 && value != 4 && value != 8) return SS_E_ARG;
    st->spec_items = (uint32_t)value;
  } else if (k == "speculate_group") {
    if (value < 0) return SS_E_ARG;
    st->spec_group = (uint64_t)value;
  } else if (k == "trace") {
    st->trace = value != 0;
  } else if (k == "trace_reset") {
    for (int c = 0; c < SS_TRACE_NCAT; ++c) {
      st->tr_sec[c] = 0.0;
      st->tr_cnt[c] = st->tr_bytes[c] = st->tr_entries[c] = 0;
    }
  } else {
    return SS_E_ARG;
  }
  return SS_OK;
}

int ss_trace_read(ss_state* st, uint32_t cat, uint64_t* launches, double* seconds, uint64_t* bytes,
                  uint64_t* entries) {
  if (!st || cat >= SS_TRACE_NCAT) return SS_E_ARG;
  if (!st->pending.empty()) {
    const int rc = sync_state(st);
    if (rc) return rc;
  }
  if (launches) *launches = st->tr_cnt[cat];
  if (seconds) *seconds = st->tr_sec[cat];
  if (bytes) *bytes = st->tr_bytes[cat];
  if (entries) *entries = st->tr_entries[cat];
  return SS_OK;
}

int ss_device_error(const ss_state* st, uint32_t* bits) {
  if (!st || !bits) return SS_E_ARG;
  *bits = st->dev_err;
  return SS_OK;
}

int ss_stats(const ss_state* st, uint64_t* out9) {
  if (!st || !out9) return SS_E_ARG;
  for (int i = 0; i < 8; ++i) out9[i] = st->stats[i];
  out9[8] = st->spec_fail_seen[0] + st->spec_fail_seen[1];
  return SS_OK;
}

}  // extern "C"
