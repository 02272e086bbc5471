"""Semblance-call counts of the two searches (host-side bookkeeping).

Used to cross-check the device's own evaluation counter.
"""
from __future__ import annotations

import math


def evals_jade(p_d: int, np_: int, ng: int) -> int:
    """Per-domain search: P_d NP (1 + NG) calls (eq. jade_semblance)."""
    return int(p_d) * int(np_) * (1 + int(ng))


def evals_ens(p_d: int, np_f: int, ng_f: int, np_bf: int, ng_bf: int, n_cycle: int,
              n_skip: int = 0) -> int:
    """ENS calls (section "ENS Semblance computations", eq. ens_semblance).

    S_f = NP_f (1 + NG_f) per estimated sample in the exploration sweep;
    S_bf = 2 (NP_bf (1 + NG_bf) - 1) per cycle (one member of each
    backward/forward population keeps its stored score); each skipped sample
    costs one more call per sweep.  The estimated samples are
    ceil(P_d / (N_skip + 1)).
    """
    s_f = int(np_f) * (1 + int(ng_f))
    s_bf = 2 * (int(np_bf) * (1 + int(ng_bf)) - 1)
    est = math.ceil(int(p_d) / (int(n_skip) + 1))
    return est * (s_f + int(n_cycle) * s_bf + (2 * int(n_cycle) + 1) * int(n_skip))
