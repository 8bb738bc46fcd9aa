"""Helpers shared by the GPU parity tests (marshalling between the oracle's
layouts and the library's, tolerances)."""
import sys

import numpy as np

from oracle import network, reconstruction as rc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def n_out(cc, i):
    return sum(1 for _, r in cc.incident(i) if r == "out")


def oracle_attributed(cc, variants):
    """Oracle entries with the 1/2-per-out-cut folded in, [4^c][2^d]."""
    return [rc.fold_half(rc.attribute(cc, i, variants[i]), n_out(cc, i)) for i in range(cc.n_sub)]


def bins_from_masks(m, d):
    """Explicit bins (lists of states) of one subcircuit's masks, bin order =
    compacted active bits ascending."""
    out = {}
    for x in range(1 << d):
        if (x & m.fixed) != m.fixed_val:
            continue
        b = 0
        j = 0
        for bit in range(d):
            if (m.active >> bit) & 1:
                b |= ((x >> bit) & 1) << j
                j += 1
        out.setdefault(b, []).append(x)
    return [out[k] for k in sorted(out)]


def error_bound(Ts, cc):
    """Sum of |terms| per output (contraction of |T|), the scale of rounding."""
    return network.contract_all([np.abs(T) for T in Ts], cc)
