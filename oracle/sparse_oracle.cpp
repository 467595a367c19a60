// Sparse register-level simulator: the ORACLE (test infrastructure only).
//
// Only tests, the smoke check and the benchmark's CPU-baseline leg load this
// library.  It shares no code, header, table or constant with the HIP path:
// it is a plain, slow, obviously correct std::map implementation of what the
// simulator computes, in double-precision complex arithmetic written out by
// hand (built with -ffp-contract=off so no product is fused into an add).
//
// What it follows (SparQSim, arXiv 2503.15118):
//  * state  sum_i a_i |v^0_i>|v^1_i>...|v^{K-1}_i>, only nonzero branches kept
//    (Sec. "Sparse state representation and data structure", its equation);
//    each register is a fixed-width binary string (same section).
//  * non-interference ops act on every branch independently; a control test
//    gates the update; no branch is created or removed
//    (Sec. "Non-interference operations").
//  * interference ops combine coherent branches (equal idle qubits), may
//    create branches, and zero-amplitude branches are removed afterwards
//    (Sec. "Interference operations"; the clear-zero step after each
//    interference op in the supplementary details of quantum operations).
//  * gate matrices H and Ry; controlled-U = |0><0| (x) I + |1><1| (x) U
//    (Sec. "Qubits and quantum operations").
//  * QRAM  U|i>_A|j>_D = |i>_A|j xor d_i>_D (QRAM section, its equation);
//    the inverse is the same map.
//  * reflection R = i(2|0><0|_anc - I_anc) (x) I (QLSS section, equation of R).
//  * Y = [[0, -i], [i, 0]], Z = diag(1, -1) (Sec. "Qubits and quantum
//    operations"); the phase gates S = diag(1, i), T = diag(1, e^{i pi/4}) and
//    their inverses, named among the non-interference ops (Sec.
//    "Non-interference operations"), and diag(1, e^{i theta});
//  * a general single-qubit rotation by a 2x2 complex matrix (Rot_Int in the
//    supplementary details of quantum operations), which there dispatches on
//    a diagonal, an off-diagonal or a general matrix;
//  * register arithmetic as oracles: add a constant, multiply, divide (Sec.
//    "Non-interference operations", quantum arithmetic).
//
// Readings where the paper is silent (all listed in the design notes):
//  * qubit q of a register is bit q of its value; registers are packed in
//    creation order into 64-bit words, first fit, never straddling a word;
//    the key orders as an unsigned integer with word 3 most significant.
//  * a branching op on several qubits is the product of single-qubit ops in
//    ascending qubit order; for each qubit the parents are visited in
//    ascending key order and, per parent, child 0 before child 1; a child
//    whose matrix element is exactly 0.0 is not created.
//  * after every branching op (never after a non-branching op) an entry is
//    removed when re*re + im*im < eps*eps, or when it is exactly zero.
//  * ADD/SUB/XOR: dst <- dst op src, src truncated to the width of dst,
//    result mod 2^width(dst).  MULC: dst <- dst*c mod 2^width, c odd.
//  * Y, Z, S, S^-1, T, T^-1, the phase gate and a rotation whose matrix is
//    diagonal or off-diagonal map every branch to one branch: they are
//    non-interference ops (no pruning after them).  On several qubits they
//    act on each qubit of the mask in ascending order.  A rotation by any
//    other matrix is an interference op on one qubit (pruned afterwards); an
//    element is "zero" when its real and imaginary parts are both 0.0.
//  * complex products are written out: (a + ib)(c + id) = (ac - bd) + i(ad + bc).
//  * ADDC: dst <- dst + c mod 2^width.  MUL: dst <- dst xor (x * y mod
//    2^width(dst)).  DIV: q <- q xor (x div y), r <- r xor (x mod y), each
//    truncated to its register; for y = 0 the quotient is all ones and the
//    remainder x (the xor form keeps both maps bijections).
//  * registers can be added and removed while the state lives (the System
//    class's add_register / remove_register, supplementary Table S1): a new
//    register takes the lowest run of free bits of its width in the lowest
//    key word that has one (a word is added when none has), every branch
//    holding 0 there; a register can be removed when it holds one value v in
//    every branch (the state is then that register's |v> times the rest), and
//    its bits are cleared.  Its index stays retired.
//  * probability readout without collapse: p(v)/P for every v with weight.
//  * measurement: p(v) = sum of |a|^2 over entries whose field equals v
//    (ascending key), P = sum of p(v) over ascending v; the outcome is the
//    smallest v whose running sum exceeds u*P; survivors are divided by
//    sqrt(p(v)); the returned probability is p(v)/P.
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

using Key = std::array<uint64_t, 4>;

struct KeyLess {
  bool operator()(const Key& x, const Key& y) const {
    for (int w = 3; w >= 0; --w) {
      if (x[w] != y[w]) return x[w] < y[w];
    }
    return false;
  }
};

struct Amp {
  double re = 0.0, im = 0.0;
};

using State = std::map<Key, Amp, KeyLess>;

enum OracleKind : uint32_t {
  K_X = 0, K_H = 1, K_RY = 2, K_ADD = 3, K_SUB = 4, K_MULC = 5, K_XOR = 6,
  K_XORC = 7, K_QLOAD = 8, K_QUNLOAD = 9, K_REFLECT0 = 10,
  K_Y = 11, K_Z = 12, K_S = 13, K_SDG = 14, K_T = 15, K_TDG = 16, K_PHASE = 17,
  K_ROT = 18, K_ADDC = 19, K_MUL = 20, K_DIV = 21
};

// A 2x2 complex matrix, m[out][in].
struct Mat {
  Amp m[2][2];
};

struct Field {
  int word;
  int offset;
  int width;    // 0: a removed register
};

struct QTable {
  std::vector<uint64_t> words;
  uint32_t addr_bits, word_bits;
};

struct Oracle {
  std::vector<Field> regs;
  double eps;
  State state;
  std::vector<QTable> tables;
  std::vector<Mat> mats;
  uint64_t peak = 0;
};

Amp cmul(const Amp& a, const Amp& b) {
  Amp r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}

bool is_zero(const Amp& a) { return a.re == 0.0 && a.im == 0.0; }

uint64_t low_mask(int width) { return width >= 64 ? ~0ull : ((1ull << width) - 1ull); }

uint64_t get_field(const Key& k, const Field& f) {
  return (k[f.word] >> f.offset) & low_mask(f.width);
}

void set_field(Key& k, const Field& f, uint64_t v) {
  uint64_t m = low_mask(f.width) << f.offset;
  k[f.word] = (k[f.word] & ~m) | ((v << f.offset) & m);
}

bool get_bit(const Key& k, const Field& f, int q) { return (k[f.word] >> (f.offset + q)) & 1ull; }

}  // namespace

extern "C" {

// Op record understood by the oracle.  Kinds follow OracleKind above.
// MUL: reg <- reg xor (reg2 * reg3).  DIV: reg (quotient) and reg4
// (remainder) from reg2 (dividend) and reg3 (divisor).  ROT: table is the
// matrix index from ora_add_matrix.
struct ora_op {
  uint32_t kind, nctl, reg, reg2, table, reg3;
  uint64_t qmask, imm;
  double theta;
  uint32_t ctl_reg[3], ctl_qubit[3], ctl_val[3];
  uint32_t reg4;
};

void* ora_create(const uint32_t* widths, uint32_t nregs, double eps) {
  Oracle* o = new Oracle();
  o->eps = eps;
  int fill[4] = {0, 0, 0, 0};
  for (uint32_t r = 0; r < nregs; ++r) {
    int w = (int)widths[r];
    if (w < 1 || w > 64) { delete o; return nullptr; }
    int word = 0;
    while (word < 4 && fill[word] + w > 64) ++word;
    if (word == 4) { delete o; return nullptr; }
    o->regs.push_back({word, fill[word], w});
    fill[word] += w;
  }
  Key zero{};
  o->state[zero] = Amp{1.0, 0.0};
  o->peak = 1;
  return o;
}

void ora_destroy(void* h) { delete static_cast<Oracle*>(h); }

// Where register r sits in the packed key (for tests of the packing rule).
int ora_layout(void* h, uint32_t r, uint32_t* word, uint32_t* offset) {
  Oracle* o = static_cast<Oracle*>(h);
  if (r >= o->regs.size()) return -1;
  *word = o->regs[r].word;
  *offset = o->regs[r].offset;
  return 0;
}

int ora_add_table(void* h, const uint64_t* vals, uint64_t len, uint32_t addr_bits,
                  uint32_t word_bits) {
  Oracle* o = static_cast<Oracle*>(h);
  if (addr_bits > 40 || len != (1ull << addr_bits)) return -1;
  QTable t;
  t.addr_bits = addr_bits;
  t.word_bits = word_bits;
  t.words.assign(vals, vals + len);
  for (uint64_t v : t.words)
    if (word_bits < 64 && (v >> word_bits) != 0) return -1;
  o->tables.push_back(std::move(t));
  return (int)o->tables.size() - 1;
}

// Add a register of `width` qubits holding 0 in every branch; returns its
// index, or -1 when no key word (of at most 4) has room.
int ora_add_register(void* h, uint32_t width) {
  Oracle* o = static_cast<Oracle*>(h);
  if (width < 1 || width > 64) return -1;
  for (int w = 0; w < 4; ++w) {
    uint64_t used = 0;
    for (const Field& f : o->regs)
      if (f.width && f.word == w) used |= low_mask(f.width) << f.offset;
    for (int off = 0; off + (int)width <= 64; ++off) {
      if ((used & (low_mask(width) << off)) == 0) {
        o->regs.push_back({w, off, (int)width});
        return (int)o->regs.size() - 1;
      }
    }
  }
  return -1;
}

// Remove register r: -1 unless it holds one value in every branch; that
// value's bits are cleared from every key.
int ora_remove_register(void* h, uint32_t r) {
  Oracle* o = static_cast<Oracle*>(h);
  if (r >= o->regs.size() || o->regs[r].width == 0) return -1;
  const Field f = o->regs[r];
  bool first = true;
  uint64_t v0 = 0;
  for (const auto& kv : o->state) {
    uint64_t v = get_field(kv.first, f);
    if (first) { v0 = v; first = false; }
    else if (v != v0) return -1;
  }
  State out;
  for (const auto& kv : o->state) {
    Key k = kv.first;
    set_field(k, f, 0);
    out[k] = kv.second;
  }
  o->state.swap(out);
  o->regs[r].width = 0;
  return 0;
}

// Probabilities of register `reg` without collapse: for each value v with
// weight (ascending), p(v) / P with p(v) the sum of |a|^2 over its branches
// (ascending key) and P the sum of p(v) (ascending v).  Writes up to `cap`
// pairs; returns the number of values.
uint64_t ora_probabilities(void* h, uint32_t reg, uint64_t* values, double* probs, uint64_t cap) {
  Oracle* o = static_cast<Oracle*>(h);
  const Field& f = o->regs[reg];
  std::map<uint64_t, double> p;
  for (const auto& kv : o->state) {
    double n2 = kv.second.re * kv.second.re + kv.second.im * kv.second.im;
    p[get_field(kv.first, f)] += n2;
  }
  double P = 0.0;
  for (const auto& pv : p) P += pv.second;
  uint64_t i = 0;
  for (const auto& pv : p) {
    if (i < cap) {
      values[i] = pv.first;
      probs[i] = pv.second / P;
    }
    ++i;
  }
  return i;
}

// Register a 2x2 complex matrix (8 doubles: m00, m01, m10, m11 as re, im;
// row = output bit) for ROT ops; returns its index.
int ora_add_matrix(void* h, const double* m8) {
  Oracle* o = static_cast<Oracle*>(h);
  Mat m;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) m.m[r][c] = Amp{m8[4 * r + 2 * c], m8[4 * r + 2 * c + 1]};
  o->mats.push_back(m);
  return (int)o->mats.size() - 1;
}

// Replace the state by the given entries (register values, row-major n x nregs).
int ora_set_entries(void* h, const uint64_t* values, const double* amps, uint64_t n) {
  Oracle* o = static_cast<Oracle*>(h);
  State s;
  size_t nr = o->regs.size();
  for (uint64_t i = 0; i < n; ++i) {
    Key k{};
    for (size_t r = 0; r < nr; ++r) set_field(k, o->regs[r], values[i * nr + r]);
    if (s.count(k)) return -1;
    s[k] = Amp{amps[2 * i], amps[2 * i + 1]};
  }
  o->state.swap(s);
  if (o->state.size() > o->peak) o->peak = o->state.size();
  return 0;
}

}  // extern "C"

namespace {

bool controls_hold(const Oracle* o, const ora_op& op, const Key& k) {
  for (uint32_t j = 0; j < op.nctl; ++j) {
    const Field& f = o->regs[op.ctl_reg[j]];
    if ((uint32_t)get_bit(k, f, (int)op.ctl_qubit[j]) != op.ctl_val[j]) return false;
  }
  return true;
}

// Non-interference op: key -> f(key), amplitude -> phase(key) * amplitude.
int apply_permutation(Oracle* o, const ora_op& op) {
  State out;
  const Field& dst = o->regs[op.reg];
  uint64_t wmask = low_mask(dst.width);
  for (const auto& kv : o->state) {
    Key k = kv.first;
    Amp a = kv.second;
    if (controls_hold(o, op, k)) {
      uint64_t v = get_field(k, dst);
      switch (op.kind) {
        case K_X: v ^= (op.qmask & wmask); break;
        case K_ADD: v = (v + get_field(k, o->regs[op.reg2])) & wmask; break;
        case K_SUB: v = (v - get_field(k, o->regs[op.reg2])) & wmask; break;
        case K_MULC: v = (v * op.imm) & wmask; break;
        case K_XOR: v = (v ^ get_field(k, o->regs[op.reg2])) & wmask; break;
        case K_XORC: v = (v ^ op.imm) & wmask; break;
        case K_QLOAD:
        case K_QUNLOAD: {
          const QTable& t = o->tables[op.table];
          uint64_t addr = get_field(k, o->regs[op.reg2]);
          v = (v ^ t.words[addr]) & wmask;
          break;
        }
        case K_REFLECT0: {
          // i * (re + i im) = -im + i re ;  -i * (re + i im) = im - i re
          Amp b;
          if (v == 0) { b.re = -a.im; b.im = a.re; }
          else        { b.re = a.im;  b.im = -a.re; }
          a = b;
          break;
        }
        case K_ADDC: v = (v + op.imm) & wmask; break;
        case K_MUL: {
          uint64_t x = get_field(k, o->regs[op.reg2]), y = get_field(k, o->regs[op.reg3]);
          v = (v ^ (x * y)) & wmask;
          break;
        }
        case K_DIV: {
          uint64_t x = get_field(k, o->regs[op.reg2]), y = get_field(k, o->regs[op.reg3]);
          const Field& rf = o->regs[op.reg4];
          uint64_t q = y ? x / y : ~0ull, r = y ? x % y : x;
          v = (v ^ q) & wmask;
          set_field(k, rf, (get_field(k, rf) ^ r) & low_mask(rf.width));
          break;
        }
        default: return -2;
      }
      set_field(k, dst, v);
    }
    if (out.count(k)) return -3;  // not a bijection
    out[k] = a;
  }
  o->state.swap(out);
  return 0;
}

// One single-qubit interference step with the real 2x2 matrix m (row = output
// bit, column = input bit); no pruning here.
void apply_single_qubit(Oracle* o, const ora_op& op, const Field& f, int q, const double m[2][2]) {
  State out;
  for (const auto& kv : o->state) {
    const Key& k = kv.first;
    const Amp& a = kv.second;
    if (!controls_hold(o, op, k)) {
      Amp& d = out[k];
      d.re = d.re + a.re;
      d.im = d.im + a.im;
      continue;
    }
    int b = get_bit(k, f, q) ? 1 : 0;
    for (int s = 0; s < 2; ++s) {
      double c = m[s][b];
      if (c == 0.0) continue;
      Key child = k;
      uint64_t bit = 1ull << (f.offset + q);
      if (s) child[f.word] |= bit; else child[f.word] &= ~bit;
      double pr = c * a.re;
      double pi = c * a.im;
      Amp& d = out[child];
      d.re = d.re + pr;
      d.im = d.im + pi;
    }
  }
  o->state.swap(out);
}

// The same step with a complex matrix (ROT): children whose matrix element
// has both parts 0.0 are not created.
void apply_single_qubit_complex(Oracle* o, const ora_op& op, const Field& f, int q, const Mat& m) {
  State out;
  for (const auto& kv : o->state) {
    const Key& k = kv.first;
    const Amp& a = kv.second;
    if (!controls_hold(o, op, k)) {
      Amp& d = out[k];
      d.re = d.re + a.re;
      d.im = d.im + a.im;
      continue;
    }
    int b = get_bit(k, f, q) ? 1 : 0;
    for (int s = 0; s < 2; ++s) {
      const Amp& c = m.m[s][b];
      if (is_zero(c)) continue;
      Key child = k;
      uint64_t bit = 1ull << (f.offset + q);
      if (s) child[f.word] |= bit; else child[f.word] &= ~bit;
      Amp p = cmul(a, c);
      Amp& d = out[child];
      d.re = d.re + p.re;
      d.im = d.im + p.im;
    }
  }
  o->state.swap(out);
}

// A single-qubit gate that keeps each branch one branch, on every qubit of
// the mask in ascending order: where the controls hold, bit b of qubit q
// becomes b ^ flip and the amplitude is multiplied by fac[b].
int apply_one_to_one(Oracle* o, const ora_op& op, bool flip, const Amp fac[2]) {
  const Field& f = o->regs[op.reg];
  for (int q = 0; q < f.width; ++q) {
    if (!((op.qmask >> q) & 1ull)) continue;
    State out;
    for (const auto& kv : o->state) {
      Key k = kv.first;
      Amp a = kv.second;
      if (controls_hold(o, op, k)) {
        int b = get_bit(k, f, q) ? 1 : 0;
        a = cmul(a, fac[b]);
        if (flip) k[f.word] ^= 1ull << (f.offset + q);
      }
      if (out.count(k)) return -3;
      out[k] = a;
    }
    o->state.swap(out);
  }
  return 0;
}

// The diagonal / off-diagonal gates: fac[b] is the matrix element that takes
// input bit b to its output bit.
int apply_phase_family(Oracle* o, const ora_op& op) {
  const double c = 0.70710678118654752440;  // cos(pi/4) = sin(pi/4) as the nearest double
  Amp fac[2] = {Amp{1.0, 0.0}, Amp{1.0, 0.0}};
  bool flip = false;
  switch (op.kind) {
    case K_Y: flip = true; fac[0] = Amp{0.0, 1.0}; fac[1] = Amp{0.0, -1.0}; break;  // m10 = i, m01 = -i
    case K_Z: fac[1] = Amp{-1.0, 0.0}; break;
    case K_S: fac[1] = Amp{0.0, 1.0}; break;
    case K_SDG: fac[1] = Amp{0.0, -1.0}; break;
    case K_T: fac[1] = Amp{c, c}; break;
    case K_TDG: fac[1] = Amp{c, -c}; break;
    case K_PHASE: fac[1] = Amp{std::cos(op.theta), std::sin(op.theta)}; break;
    default: return -2;
  }
  return apply_one_to_one(o, op, flip, fac);
}

void prune(Oracle* o, double eps) {
  double e2 = eps * eps;
  for (auto it = o->state.begin(); it != o->state.end();) {
    double re = it->second.re, im = it->second.im;
    double n2 = re * re + im * im;
    if (n2 < e2 || (re == 0.0 && im == 0.0)) it = o->state.erase(it);
    else ++it;
  }
}

int apply_branching(Oracle* o, const ora_op& op) {
  const Field& f = o->regs[op.reg];
  double m[2][2];
  if (op.kind == K_H) {
    // H = (1/sqrt 2) [[1, 1], [1, -1]]; 1/sqrt(2) as the nearest double.
    const double c = 0.70710678118654752440;
    m[0][0] = c; m[0][1] = c; m[1][0] = c; m[1][1] = -c;
  } else {
    // Ry(theta) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]].
    double h = op.theta / 2.0;
    double c = std::cos(h), s = std::sin(h);
    m[0][0] = c; m[0][1] = -s; m[1][0] = s; m[1][1] = c;
  }
  for (int q = 0; q < f.width; ++q) {
    if ((op.qmask >> q) & 1ull) apply_single_qubit(o, op, f, q, m);
  }
  prune(o, o->eps);
  return 0;
}

}  // namespace

extern "C" {

// Apply ops in order.  *seconds gets the wall time of the op loop alone
// (steady clock) and *entries_in the sum over ops of the input entry count.
int ora_apply(void* h, const ora_op* ops, uint64_t nops, double* seconds, uint64_t* entries_in) {
  Oracle* o = static_cast<Oracle*>(h);
  uint64_t ein = 0;
  auto t0 = std::chrono::steady_clock::now();
  for (uint64_t i = 0; i < nops; ++i) {
    const ora_op& op = ops[i];
    ein += o->state.size();
    if (o->state.empty()) continue;
    int rc;
    if (op.kind == K_H || op.kind == K_RY) {
      rc = apply_branching(o, op);
    } else if (op.kind >= K_Y && op.kind <= K_PHASE) {
      rc = apply_phase_family(o, op);
    } else if (op.kind == K_ROT) {
      if (op.table >= o->mats.size()) return -4;
      const Mat& m = o->mats[op.table];
      if (is_zero(m.m[0][1]) && is_zero(m.m[1][0])) {
        const Amp fac[2] = {m.m[0][0], m.m[1][1]};
        rc = apply_one_to_one(o, op, false, fac);
      } else if (is_zero(m.m[0][0]) && is_zero(m.m[1][1])) {
        const Amp fac[2] = {m.m[1][0], m.m[0][1]};
        rc = apply_one_to_one(o, op, true, fac);
      } else {
        const Field& f = o->regs[op.reg];
        for (int q = 0; q < f.width; ++q)
          if ((op.qmask >> q) & 1ull) apply_single_qubit_complex(o, op, f, q, m);
        prune(o, o->eps);
        rc = 0;
      }
    } else {
      rc = apply_permutation(o, op);
    }
    if (rc) return rc;
    if (o->state.size() > o->peak) o->peak = o->state.size();
  }
  auto t1 = std::chrono::steady_clock::now();
  if (seconds) *seconds = std::chrono::duration<double>(t1 - t0).count();
  if (entries_in) *entries_in = ein;
  return 0;
}

int ora_prune(void* h, double eps) {
  prune(static_cast<Oracle*>(h), eps);
  return 0;
}

int ora_measure(void* h, uint32_t reg, double u, uint64_t* outcome, double* prob) {
  Oracle* o = static_cast<Oracle*>(h);
  if (reg >= o->regs.size() || o->state.empty()) return -1;
  const Field& f = o->regs[reg];
  std::map<uint64_t, double> p;
  for (const auto& kv : o->state) {
    double n2 = kv.second.re * kv.second.re + kv.second.im * kv.second.im;
    p[get_field(kv.first, f)] += n2;
  }
  double P = 0.0;
  for (const auto& pv : p) P += pv.second;
  double target = u * P, run = 0.0;
  uint64_t v = p.rbegin()->first;
  double pv_sel = p.rbegin()->second;
  for (const auto& pv : p) {
    run += pv.second;
    if (run > target) { v = pv.first; pv_sel = pv.second; break; }
  }
  double s = std::sqrt(pv_sel);
  State out;
  for (const auto& kv : o->state) {
    if (get_field(kv.first, f) != v) continue;
    out[kv.first] = Amp{kv.second.re / s, kv.second.im / s};
  }
  o->state.swap(out);
  *outcome = v;
  *prob = pv_sel / P;
  return 0;
}

uint64_t ora_nnz(void* h) { return static_cast<Oracle*>(h)->state.size(); }
uint64_t ora_peak(void* h) { return static_cast<Oracle*>(h)->peak; }

// Entries in ascending key order: packed key (4 words each), register values
// (nregs each) and amplitudes (re, im).  Returns the number written.
uint64_t ora_export(void* h, uint64_t* keys, uint64_t* values, double* amps, uint64_t cap) {
  Oracle* o = static_cast<Oracle*>(h);
  size_t nr = o->regs.size();
  uint64_t i = 0;
  for (const auto& kv : o->state) {
    if (i >= cap) break;
    for (int w = 0; w < 4; ++w) keys[4 * i + w] = kv.first[w];
    for (size_t r = 0; r < nr; ++r) values[i * nr + r] = get_field(kv.first, o->regs[r]);
    amps[2 * i] = kv.second.re;
    amps[2 * i + 1] = kv.second.im;
    ++i;
  }
  return i;
}

}  // extern "C"
