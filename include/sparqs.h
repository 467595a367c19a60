/* sparqs: sparse register-level quantum-state simulator, hot path on one AMD
 * MI355X (gfx950).  C ABI.
 *
 * The method (SparQSim, arXiv 2503.15118) keeps a quantum state only as its
 * nonzero branches: pairs (basis key, complex amplitude), where the key is the
 * concatenation of register values (Sec. "Sparse state representation and data
 * structure", its equation for |psi>).  Non-interference ops rewrite every
 * branch independently (Sec. "Non-interference operations"); interference ops
 * sort branches so coherent ones (equal idle qubits) sit together, combine each
 * group with the gate matrix, and drop zero-amplitude branches (Sec.
 * "Interference operations" and the supplementary details of Rot_Int and
 * ClearZero).  QRAM is U|i>_A|j>_D = |i>_A|j xor d_i>_D (QRAM section, its
 * equation); R = i(2|0><0|_anc - I) (x) I is the walk's reflection (QLSS
 * section).
 *
 * Conventions used by every call:
 *  - Qubit q of a register is bit q of its value (LSB = qubit 0).
 *  - Registers (1..64 qubits each) are packed in creation order into 64-bit
 *    key words, first fit, never straddling a word; W (1, 2 or 4) words per
 *    key.  With ninst > 1 an instance-id field follows the registers (first
 *    fit as well); keys handed out by ss_export have that field cleared.
 *  - Keys order as unsigned integers with word W-1 most significant.
 *  - Amplitudes are complex128, passed as interleaved (re, im) doubles.
 *  - After every branching op (H, RY), never after a non-branching op, an
 *    entry is removed when re*re + im*im < eps*eps or when it is exactly 0.
 *
 * Memory and threads: the caller owns the device arena (e.g. a torch uint8
 * CUDA tensor) and the HIP stream; the library never allocates device memory
 * (it allocates one small pinned host block per state for read-back).  Input
 * arrays are copied before a call returns; no caller pointer is retained.  A
 * state may be used by one host thread at a time; distinct states are
 * independent.
 *
 * Errors: every call returns SS_OK (0) or a negative SS_E_* code; nothing is
 * thrown across the ABI.  A state that hit SS_E_HIP is poisoned and further
 * calls return SS_E_STATE.
 */
#ifndef SPARQS_H
#define SPARQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ss_status {
  SS_OK = 0,
  SS_E_ARG = -1,          /* bad register/qubit/instance, dst == src, control inside dst, empty mask */
  SS_E_NOT_UNITARY = -2,  /* even MULC constant */
  SS_E_QRAM = -3,         /* table length != 2^addr_bits, entry too wide, width mismatch */
  SS_E_CAPACITY = -4,     /* an op would exceed the arena's entry capacity (state rolled back) */
  SS_E_NOMEM = -5,        /* arena too small at creation */
  SS_E_HIP = -6,          /* HIP runtime or kernel-side failure; the state is poisoned */
  SS_E_STATE = -7,        /* use of a poisoned or null state */
  SS_E_PLAN = -8          /* a graph replay met a state its captured plan does not fit (rolled back) */
};

enum ss_kind {
  SS_X = 0,           /* flip the qubits of qmask in reg (CNOT/Toffoli via controls) */
  SS_H = 1,           /* Hadamard on each qubit of qmask, ascending */
  SS_RY = 2,          /* Ry(theta) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]] on each qubit of qmask */
  SS_ADD = 3,         /* reg <- reg + reg2 mod 2^width(reg) */
  SS_SUB = 4,         /* reg <- reg - reg2 mod 2^width(reg) */
  SS_MULC = 5,        /* reg <- reg * imm mod 2^width(reg), imm odd */
  SS_XOR = 6,         /* reg <- reg xor reg2 (truncated to width(reg)) */
  SS_XORC = 7,        /* reg <- reg xor imm (truncated) */
  SS_QRAM_LOAD = 8,   /* reg (data) <- reg xor table[reg2 (address)] */
  SS_QRAM_UNLOAD = 9, /* the inverse, the same map */
  SS_REFLECT0 = 10,   /* amplitude *= +i if reg == 0 else -i */
  /* Gates that keep each branch one branch (non-interference ops, never
   * followed by a prune), on each qubit of qmask in ascending order: */
  SS_Y = 11,          /* Y = [[0, -i], [i, 0]] */
  SS_Z = 12,          /* Z = diag(1, -1) (CZ: Z with a control) */
  SS_S = 13,          /* S = diag(1, i) */
  SS_SDG = 14,        /* S^-1 = diag(1, -i) */
  SS_T = 15,          /* T = diag(1, e^{i pi/4}), e^{i pi/4} = (c, c), c the double nearest 1/sqrt 2 */
  SS_TDG = 16,        /* T^-1 = diag(1, (c, -c)) */
  SS_PHASE = 17,      /* diag(1, cos theta + i sin theta) (host libm) */
  /* The 2x2 complex matrix aux (from ss_load_matrix) on the single qubit of
   * qmask: a diagonal or off-diagonal matrix keeps each branch one branch (no
   * prune); any other is an interference op (grouped, combined, pruned). */
  SS_ROT = 18,
  SS_ADDC = 19,       /* reg <- reg + imm mod 2^width(reg) */
  SS_MUL = 20,        /* reg <- reg xor (reg2 * aux mod 2^width(reg)); aux = a register */
  /* reg <- reg xor (reg2 div aux), imm (a register index) <- imm xor (reg2 mod
   * aux), each truncated to its register; for aux = 0 the quotient is all
   * ones and the remainder reg2 */
  SS_DIV = 21
};

typedef struct ss_reg {
  uint32_t nqubits;       /* 1..64 */
  const char* name;       /* may be NULL; informational only */
} ss_reg;

typedef struct ss_ctl {
  uint32_t reg;
  uint16_t qubit;
  uint16_t value;         /* 0 or 1: the op acts where this qubit has this value */
} ss_ctl;

/* One register-level operation, 64 bytes. */
typedef struct ss_op {
  uint16_t kind;          /* enum ss_kind */
  uint8_t nctl;           /* 0..3 controls */
  uint8_t flags;          /* must be 0 */
  uint32_t reg;           /* target / destination register */
  uint32_t reg2;          /* source register (ADD/SUB/XOR/MUL/DIV) or address register (QRAM) */
  uint32_t aux;           /* QRAM: table id (ss_load_qram); ROT: matrix id (ss_load_matrix);
                             MUL: second factor register; DIV: divisor register */
  uint64_t qmask;         /* qubits of reg (X, H, RY, Y, Z, S, SDG, T, TDG, PHASE, ROT) */
  uint64_t imm;           /* MULC multiplier, XORC / ADDC constant, DIV remainder register */
  double theta;           /* RY / PHASE angle */
  ss_ctl ctl[3];
} ss_op;

typedef struct ss_result {
  int32_t status;         /* last error, SS_OK if none */
  uint32_t failed_inst;
  uint64_t failed_op;     /* index of the op that failed (SS_E_CAPACITY: resume from here) */
  uint64_t nnz;           /* entries after the call (all instances) */
  uint64_t peak;          /* running maximum of nnz */
} ss_result;

typedef struct ss_state ss_state;

/* Device bytes an arena needs for `cap_entries` entries of this layout plus
 * `table_bytes` of QRAM tables.  Entries cost 2*(8W+16) bytes (state and its
 * alternate buffer) plus look-back scratch.
 * Defined by: the paper is silent; this is the footprint model behind
 * admission by predicted peak memory (memory is dominated by the branch
 * list, Sec. "Sparse state representation and data structure").  It takes an
 * entry capacity rather than (peak nnz, fan-out): a caller that knows a peak
 * and the widest fan-out of its ops passes peak * 2^fanout, and the same
 * capacity is what ss_create_state will carve.
 * Errors: SS_E_ARG (bad registers, null output). */
int ss_required_bytes(const ss_reg* regs, uint32_t nregs, uint32_t ninst, uint64_t cap_entries,
                      uint64_t table_bytes, size_t* bytes);

/* Create a state of `ninst` instances, each |0...0> with amplitude 1, in the
 * caller's device arena [arena, arena + arena_bytes) (256-byte aligned) on
 * `hip_stream` (a hipStream_t, NULL = default stream).  `table_bytes` of the
 * arena are reserved for QRAM tables (an argument the paper's problem
 * statement does not need; it fixes where the tables end and the entry
 * buffers begin, so the capacity is known at creation).  Blocking.
 * Defined by: the state |psi> = sum_i a_i |v^0_i>...|v^{K-1}_i> with each
 * register a fixed-width binary string (Sec. "Sparse state representation
 * and data structure", its equation); the registers are given up front.
 * Errors: SS_E_ARG (bad registers, more than 256 key bits, ninst == 0),
 * SS_E_NOMEM (arena too small for the instances), SS_E_HIP. */
int ss_create_state(const ss_reg* regs, uint32_t nregs, uint32_t ninst, double eps, void* arena,
                    size_t arena_bytes, uint64_t table_bytes, void* hip_stream, ss_state** out);

/* ss_create_state for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * state, but its scratch (meta block, digit starts, op ring, instance
 * scratch, radix histograms, look-back words) lives in a 64 MiB device array
 * inside the library, one per GPU, held until the process ends; the caller's
 * `entries` memory (256-byte aligned) holds only the QRAM tables and the two
 * entry buffers (table_bytes + 2 x capacity x (8W + 16) bytes, the capacity
 * being the largest multiple of 256 that fits both).  The call and the state
 * allocate no device or pinned host memory (host read-back and op staging are
 * static arrays); the "trace" option and ss_graph_capture still allocate.
 * One such state may live per GPU at a time: while it lives another call on
 * that GPU returns SS_E_STATE (its array holds the first state's scratch).
 * The device is the current one.  ss_rebind_arena and key growth in
 * ss_add_register are refused (SS_E_ARG, SS_E_NOMEM): the carve is fixed.
 * Errors: as ss_create_state; SS_E_NOMEM when the capacity that the 64 MiB
 * scratch or the entry memory allows is below max(256, ninst). */
int ss_create_state_noalloc(const ss_reg* regs, uint32_t nregs, uint32_t ninst, double eps, void* entries,
                            size_t entry_bytes, uint64_t table_bytes, void* hip_stream, ss_state** out);

/* Free host-side metadata (and the state's pinned read-back block) after
 * waiting for the stream; the arena stays the caller's.  SS_E_STATE for a
 * null state. */
int ss_destroy_state(ss_state* st);

/* Entry capacity of the arena (all instances together). */
int ss_capacity(const ss_state* st, uint64_t* cap);

/* Where register `reg` sits in the key: word index, bit offset, width. */
int ss_layout(const ss_state* st, uint32_t reg, uint32_t* word, uint32_t* offset, uint32_t* width);

/* Key words per entry (1, 2 or 4). */
int ss_key_words(const ss_state* st, uint32_t* w);

/* Copy a QRAM table (host array of `len` words) into the arena.  Requires
 * len == 2^addr_bits and every word < 2^word_bits (SS_E_QRAM otherwise;
 * SS_E_NOMEM when the reserved table bytes are used up).  *qram_id names it in
 * SS_QRAM_LOAD / SS_QRAM_UNLOAD ops.  Blocking.
 * Defined by: U_QRAM |i>_A |j>_D = |i>_A |j xor d_i>_D, with address length =
 * width of A and word length = width of D (QRAM section, its equation). */
int ss_load_qram(ss_state* st, const uint64_t* table, uint64_t len, uint32_t addr_bits,
                 uint32_t word_bits, uint32_t* qram_id);

/* Register a 2x2 complex matrix for SS_ROT ops: m = 8 doubles, the elements
 * m00, m01, m10, m11 (row = output bit, column = input bit) each as (re, im).
 * The matrix must be unitary to within 1e-12 (max-norm of M^H M - I), else
 * SS_E_NOT_UNITARY; *matrix_id names it in ops.  Host-side only (the values
 * travel in each op's launch arguments).
 * Defined by: the general rotation on a single qubit by a 2x2 matrix (Rot_Int
 * in the supplementary details of quantum operations), with the controlled
 * form CU = |0><0| (x) I + |1><1| (x) U (Sec. "Qubits and quantum
 * operations"). */
int ss_load_matrix(ss_state* st, const double* m, uint32_t* matrix_id);

/* Replace the entries of instance `inst` by n entries given as register values
 * (host, row-major n x nregs) and amplitudes (host, 2n doubles).  Values are
 * truncated to the register widths.  Register values rather than packed keys
 * are taken so that callers need not know the packing (ss_layout reports it).
 * Errors: SS_E_ARG (bad instance, null arrays, two entries with the same
 * key: checked before anything changes), SS_E_CAPACITY (the state keeps the
 * other instances' entries; this instance is then empty).  Blocking.
 * Defined by: the state equation of Sec. "Sparse state representation and
 * data structure" (one amplitude per distinct basis key). */
int ss_set_entries(ss_state* st, uint32_t inst, const uint64_t* values, const double* amps, uint64_t n);

/* Apply `nops` ops.  With inst_offsets == NULL every instance gets the same
 * ops.  Returns when the work is done (the status is final).  On
 * SS_E_CAPACITY the state holds the result of ops [0, res->failed_op) and the
 * caller may rebind a larger arena and resume from failed_op.
 * Errors: SS_E_ARG (a bad op: register, qubit, dst == src, a control inside
 * dst, an empty mask, ROT on more than one qubit or an unknown matrix;
 * nothing applied), SS_E_NOT_UNITARY, SS_E_QRAM, SS_E_CAPACITY, SS_E_HIP.
 * Defined by: non-branching kinds (X and its controlled forms, ADD, SUB,
 * MULC, XOR, XORC, QRAM, ADDC, MUL, DIV, the Pauli and phase gates Y, Z, S,
 * T and their inverses) rewrite each branch on its own (Sec.
 * "Non-interference operations"; Y and Z as in Sec. "Qubits and quantum
 * operations"); ROT dispatches on its matrix as Rot_Int does (supplementary
 * details of quantum operations); the QRAM kinds follow the QRAM section's
 * equation; REFLECT0 is R = i(2|0><0|_anc - I) (x) I of the QLSS section;
 * H and RY group coherent branches, combine each group with the gate matrix
 * (Sec. "Qubits and quantum operations" for the matrices, controlled-U =
 * |0><0| (x) I + |1><1| (x) U) and then drop zero branches (Sec.
 * "Interference operations"; ClearZero after Rot_Int in the supplementary
 * details of quantum operations). */
int ss_apply_ops(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* inst_offsets,
                 ss_result* res);

/* Remove entries with |a|^2 < eps^2 or a == 0 (eps >= 0, else SS_E_ARG).
 * Blocking.
 * Defined by: the zero-branch removal after interference ops (Sec.
 * "Interference operations"; ClearZero in the supplementary details of
 * quantum operations), with the paper's "zero" read as |a| < eps. */
int ss_prune(ss_state* st, double eps);

/* Collapsing measurement of register `reg` of instance `inst` with the caller's
 * uniform draw u in [0, 1): p(v) = sum of |a|^2 over entries with field v,
 * P = sum over v; the outcome is the smallest v whose running sum (ascending
 * v) exceeds u*P (the largest v with weight if rounding leaves none); the
 * survivors are divided by sqrt(p(v)); *prob = p(v)/P.
 * Errors: SS_E_ARG (bad instance or register, u outside [0, 1), an empty
 * instance).  Blocking.
 * Defined by: the paper is silent on measurement; this is the textbook
 * projective measurement of one register in the computational basis, on the
 * state of Sec. "Sparse state representation and data structure". */
int ss_measure(ss_state* st, uint32_t inst, uint32_t reg, double u, uint64_t* outcome, double* prob);

/* Probabilities of register `reg` in instance `inst` without collapse: for
 * each value v with weight, ascending, values[k] = v and probs[k] = p(v)/P,
 * with p(v) the sum of |a|^2 over the instance's entries whose field is v and
 * P the instance's total (both summed on the device in a fixed order).
 * Writes min(cap, count) pairs; *n gets the count.  The state is unchanged
 * (its entries are left ordered by the field).  Blocking.
 * Errors: SS_E_ARG (bad instance or register, null outputs).
 * Defined by: the paper is silent on readout; this is the marginal
 * distribution of one register of the state of Sec. "Sparse state
 * representation and data structure". */
int ss_probabilities(ss_state* st, uint32_t inst, uint32_t reg, uint64_t* values, double* probs, uint64_t cap,
                     uint64_t* n);

/* Add a register of `nqubits` (1..64) qubits, |0> in every branch, to a live
 * state; *reg gets its index (indices of removed registers are not reused).
 * It takes the lowest run of free key bits of its width in the lowest key word
 * that has one (bits freed by removed registers included).  When no word has
 * room the key gains words (W 1 -> 2 -> 4): the entries are re-packed on the
 * device inside the same arena, whose entry capacity then shrinks
 * (SS_E_NOMEM, state unchanged, if the entries would not fit).  Graphs
 * captured before the call are retired.  Blocking.
 * Errors: SS_E_ARG (width, 64 registers already), SS_E_NOMEM (no room in 256
 * key bits, or the arena after re-packing).
 * Defined by: add_register of the System class (supplementary Table S1):
 * activating a register (Sec. "Sparse state representation and data
 * structure"). */
int ss_add_register(ss_state* st, uint32_t nqubits, const char* name, uint32_t* reg);

/* Remove register `reg`.  Allowed only when it holds one value v in every
 * branch of every instance (the state is then |v> on that register times the
 * rest); its bits are cleared and freed, its index retired (ops naming it
 * fail with SS_E_ARG).  Blocking.
 * Errors: SS_E_ARG (bad or removed register, more than one value).
 * Defined by: remove_register of the System class (supplementary Table S1):
 * deactivating a register. */
int ss_remove_register(ss_state* st, uint32_t reg);

/* Entry count of instance `inst` (UINT32_MAX: all instances) and the running
 * peak of the whole state (the paper's max_system_size, supplementary Table
 * S1).  Blocking. */
int ss_nnz(ss_state* st, uint32_t inst, uint64_t* nnz, uint64_t* peak);

/* Copy instance `inst`'s entries to host arrays in ascending key order:
 * keys (W words per entry, instance field cleared) and amps (2 doubles per
 * entry).  Writes min(cap, nnz) entries; *n gets nnz.  Blocking.
 * Defined by: the branch list of Sec. "Sparse state representation and data
 * structure"; the ascending order is a canonical choice (the paper keeps
 * branches in the order its sorts leave them). */
int ss_export(ss_state* st, uint32_t inst, uint64_t* keys, double* amps, uint64_t cap, uint64_t* n);

/* Wait for the stream and report kernel-side errors. */
int ss_sync(ss_state* st, ss_result* res);

/* Captured op lists (HIP graphs).
 *
 * The planner's choices for an op list (sort or not, which key bits a sort
 * covers, grid sizes) depend on entry counts and key masks that it reads back
 * from the device between launches.  ss_graph_capture applies the ops to the
 * state exactly as ss_apply_ops does (same arguments, same result, same
 * errors), recording each read-back, and then builds a HIP graph of the same
 * launch sequence, with the recorded values in place of the read-backs.  The
 * graph holds every kernel and op-record copy of the list; a replay has no
 * host synchronisation until its end.
 *
 * A replay is valid for a state on which the planner would make the same
 * choices.  At every point where the capture read back, the graph checks on
 * the device that the entry count equals the recorded one and that no key
 * bit varies that did not vary then; the first failed check makes every later
 * launch of the replay a no-op.  So a replay gives the result of
 * ss_apply_ops on the same ops, or SS_E_PLAN.
 *
 * Typical use: a circuit applied again and again to states of one shape (a
 * reset followed by the same ops, a repeated walk step).  Graphs belong to
 * their state: destroy them before the state (a graph of a destroyed state,
 * or of a state moved by ss_rebind_arena, is refused with SS_E_STATE /
 * SS_E_ARG).  Option changes after a capture do not affect the graph. */
typedef struct ss_graph ss_graph;

/* Apply `nops` ops (as ss_apply_ops) and capture them.  On success *out gets
 * the graph; on any error no graph is made, *out is NULL and the status and
 * state are those of ss_apply_ops.  SS_E_HIP here from the capture itself
 * (graph instantiation) leaves the state usable.  Blocking. */
int ss_graph_capture(ss_state* st, const ss_op* ops, uint64_t nops, const uint64_t* inst_offsets,
                     ss_result* res, ss_graph** out);

/* Replay a captured op list on its state.  Blocking, like ss_apply_ops.
 * SS_E_PLAN: the state did not fit the plan; when found before the first
 * launch (entry count differs from the capture's input) nothing ran and
 * res->failed_op = 0; otherwise the state holds the result of ops
 * [0, res->failed_op) (batched lists: rounds) and the caller may continue with
 * ss_apply_ops from there.  A divergence inside an op split over several
 * launches (H on more than 5 qubits) leaves nothing to return to: the state is
 * then poisoned.  SS_E_CAPACITY as for ss_apply_ops. */
int ss_graph_launch(ss_graph* g, ss_result* res);

/* Free the graph (host objects and its pinned op records). */
int ss_graph_destroy(ss_graph* g);

/* Move the state into another (larger) arena; the old one may be freed after
 * the call returns.  Blocking. */
int ss_rebind_arena(ss_state* st, void* arena, size_t arena_bytes);

/* Tuning/debug knobs: "sort_items" (8|16), "grouping" (1: reuse grouped
 * order across ops, 0: always sort), "group_items" (1|2|4, default 4; group-mode launches that
 * carry a chain or a run use at most 2, and the compacting launch after a
 * speculative one always 4), "perm_entries"
 * (4|8|16), "tile_order" (1: per-XCD tile tickets when the device allows,
 * taken in chunks of 8 consecutive tiles by the radix passes; 0: one
 * counter; required when states run concurrently on one GPU), "speculate" (an
 * entry count, default 2^23, 0 = never: a one-target expansion on at least
 * that many entries first places both children of every entry at fixed
 * positions, and the compacting launch after it redoes the op only when some
 * entry does not have two children; results are identical either way),
 * "chain" (1, default: up to 16 consecutive H / Ry ops on the same single
 * target qubit run as one launch in which each group gets the product of the
 * matrices whose controls hold for it, pruned once after the last; fewer when
 * eps > 1e-12/(15 sqrt 2), so that the prunes left out move no amplitude by
 * more than 1e-12; 0: one launch per op; results agree within 1e-12 and the
 * prune band),
 * "fuse_runs" (default 4096, the longest run one launch takes; 0 = never: a
 * one-target op whose next ops form a run of at most that many non-branching
 * ops applies the run to its outputs in the same launch; results are
 * identical either way),
 * "retire" (1 default, 0 off: batched calls relabel the instances by the
 * round of their last op and leave finished instances out of later rounds;
 * the labels are restored before the call returns, also after a capacity
 * failure, and results are identical either way; afterwards the entries are
 * ordered by that relabelling, not by instance),
 * "speculate_group" (as "speculate" for one-target ops on grouped entries,
 * default 2^21; there a merge or an entry without its partner defeats the
 * fixed placement, so after a wasted speculative launch the next 64
 * eligible launches of the same mode (group or expand) skip themselves, and
 * after a read-back that sees it the next 64 eligible ops of that mode do not
 * speculate, twice as many each time this repeats), "spec_items" (1|2|4|8, default 4: entries per thread of the
 * speculative launch; 8 applies to group-mode launches with a fused run and
 * lane-pair partners, the others then take 4), "pair_exchange" (how a speculative group-mode launch
 * finds partners: 2, default, only at e ^ 1 through a lane-pair exchange, a
 * tile without that alignment defeating the speculation; 1 the same with
 * staging as fallback; 0 always by staging the tile's neighbours in LDS;
 * results are identical either way), "expand_slots"
 * (1, default: an expansion on 2..5 target qubits runs one thread per child,
 * so that consecutive lanes write consecutive outputs; 0: one thread per
 * entry and its children), "trace" (1: time
 * every kernel launch with a HIP event pair on the state's stream),
 * "trace_reset". */
int ss_set_option(ss_state* st, const char* key, int64_t value);

/* Kernel categories of the trace. */
enum ss_trace_cat {
  SS_TRACE_PERM = 0,       /* fused non-branching run */
  SS_TRACE_SORT_HIST = 1,  /* radix-sort digit histograms (all passes) */
  SS_TRACE_SORT_PASS = 2,  /* one LSD scatter pass */
  SS_TRACE_GROUP = 3,      /* interference op on grouped entries */
  SS_TRACE_EXPAND = 4,     /* interference op where every group has one member */
  SS_TRACE_FILTER = 5,     /* prune / collapse compaction */
  SS_TRACE_NCAT = 6
};

/* Totals of the traced launches of one category since the last
 * "trace_reset": launch count, summed event durations (s), algorithmic bytes
 * (entries read and written at 8W+16 bytes each; a permutation run reads W
 * words and writes the touched ones, plus 32 bytes when it has a phase op)
 * and entries processed.  Blocks until pending events have completed. */
int ss_trace_read(ss_state* st, uint32_t cat, uint64_t* launches, double* seconds, uint64_t* bytes,
                  uint64_t* entries);

/* Counters since creation (out9: 9 words): [0] kernels launched, [1] sort
 * passes, [2] sorts, [3] group launches, [4] expand launches, [5] permutation
 * runs, [6] host syncs, [7] entries updated (sum over ops of input nnz),
 * [8] speculative placements that did not fit and were redone by compaction
 * (as of the last read-back). */
int ss_stats(const ss_state* st, uint64_t* out9);

/* Kernel-side error bits seen so far (diagnostics after SS_E_HIP): 1 = a
 * branching op's survivors exceeded the capacity, 2 = a tile wait gave up,
 * 4 = two entries of one group shared a target value. */
int ss_device_error(const ss_state* st, uint32_t* bits);

const char* ss_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPARQS_H */
