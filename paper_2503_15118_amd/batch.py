"""Batching: many instances with their own op lists in one state.

Each instance is a register-level circuit of the same register layout; the
state keys carry an instance-id field, and one call to ``ss_apply_ops`` with
per-instance op offsets runs every instance in rounds (one fused launch for
the non-branching ops of all instances, then one expansion / sort /
reduce-by-key for the branching ops).  Argument marshalling only.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import _abi


def concat_ops(circuits) -> tuple:
    """(ops as ss_op records, ninst + 1 offsets)."""
    parts = [_abi.to_ss_ops(c.ops) for c in circuits]
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(p) for p in parts])
    ops = np.concatenate(parts) if parts else np.zeros(0, dtype=_abi.SS_OP)
    return ops, off


def batch_state(circuits, cap_entries: int, table_bytes: int = 1 << 20, **kw) -> "_abi.State":
    """A state holding every circuit as one instance (same registers, eps and
    QRAM tables and rotation matrices, which the first circuit supplies)."""
    c0 = circuits[0]
    for c in circuits:
        if list(c.regs) != list(c0.regs):
            raise ValueError("batched instances need one register layout")
    st = _abi.State(c0.regs, ninst=len(circuits), eps=c0.eps, cap_entries=cap_entries,
                    table_bytes=table_bytes, **kw)
    for t in c0.tables:
        st.load_qram(t)
    for m in c0.matrices:
        st.load_matrix(m)
    for i, c in enumerate(circuits):
        if c.init_values is not None:
            st.set_entries(i, c.init_values, c.init_amps)
    return st


def run_batched(circuits, cap_entries: int, state: Optional["_abi.State"] = None, **kw):
    """Run every circuit as its own instance in one batched call."""
    st = state if state is not None else batch_state(circuits, cap_entries, **kw)
    ops, off = concat_ops(circuits)
    res = st.apply(ops, inst_offsets=off)
    return st, res


def run_sequential(circuits, cap_entries: int, **kw) -> List[tuple]:
    """The plain path, one instance at a time (the baseline batching is
    compared with); returns per-instance (keys, amps)."""
    out = []
    st = None
    for c in circuits:
        if st is None:
            st = _abi.state_for_circuit(c, cap_entries=cap_entries, **kw)
        else:
            zero = np.zeros((1, len(c.regs)), dtype=np.uint64)
            if c.init_values is not None:
                st.set_entries(0, c.init_values, c.init_amps)
            else:
                st.set_entries(0, zero, np.array([1.0 + 0j]))
        st.apply(c.ops)
        out.append(st.export())
    return out
