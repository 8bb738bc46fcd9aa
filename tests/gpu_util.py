"""Helpers shared by the GPU parity tests (marshalling between the oracle's
layouts and the library's, tolerances)."""
import sys

import numpy as np

from oracle import network, reconstruction as rc

# Relative factor of the a-priori rounding bound per contraction path
# (0 = FP64, 1 = FP32 MFMA, 2 = split-BF16x3): a bin computed as a sum of
# products of the entries T_i is off by at most TOL_REL * sum_sigma prod_i
# |T_i[sigma, x_i]|.  FP32 accumulation over the plan's steps costs a small
# multiple of 2^-24 per term; split-BF16x3 drops lo*lo and keeps each
# operand to 2^-16 relative, so each product is good to about 3 * 2^-16.
TOL_REL = {0: 1e-13, 1: 2.0 ** -20, 2: 2.0 ** -13}
# The absolute tolerances stated for physical data (probabilities <= 1).
TOL_ABS = {0: 1e-12, 1: 1e-6, 2: 1e-6}


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


def sampled_bound(Ts, cc, bins):
    """The same sum of |terms| at selected subcircuit-major outputs only."""
    return network.eval_bins([np.abs(T) for T in Ts], cc, bins)


def bound_tol(prec, bound, ref, bins_f32):
    """Per-bin tolerance: the path's a-priori bound, plus the rounding of the
    stored bin when bins are FP32."""
    tol = TOL_REL[prec] * np.asarray(bound, dtype=np.float64)
    if bins_f32:
        tol = tol + 2.0 ** -24 * np.abs(ref)
    return tol + 1e-300


def bound_violations(got, want, bound, prec, bins_f32):
    """Indices where |got - want| exceeds the per-bin tolerance (NaN counts)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    ok = np.abs(got - want) <= bound_tol(prec, bound, want, bins_f32)
    return np.flatnonzero(~ok)


def assert_bound(got, want, bound, prec, bins_f32, what="", physical=True):
    """Every bin within its a-priori bound, and (physical data) within the
    absolute tolerance."""
    bad = bound_violations(got, want, bound, prec, bins_f32)
    err = np.abs(np.asarray(got, dtype=np.float64) - want)
    rel = err / bound_tol(prec, bound, want, bins_f32)
    say(f"  {what}: max-abs {err.max():.3e}, max err / bound-tol {rel.max():.3f} over {len(err)} bins")
    assert len(bad) == 0, (what, bad[:8], err[bad[:8]])
    if physical:
        assert err.max() <= TOL_ABS[prec], (what, err.max())
