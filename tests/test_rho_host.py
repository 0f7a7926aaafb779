"""Section 5's speed ratio (eq. 5.1) on the host, CPU only: seconds per
CP_ALS sweep with Algorithm 1 gradients over seconds per fast sweep (Algorithm
2 inside the Section 4 loop), both float64 NumPy from the oracle package, on
small random tensors.  The paper reports the fast sweep winning and the
ratio growing with the order N (Table 5.1: about 20-30 at N = 5, 6; 42.2 for
the 7-D example); the test checks that shape of the claim, and prints the
ratios."""
import pytest

from oracle import rho_table


@pytest.mark.slow
def test_fast_sweep_wins_and_gains_with_order():
    out = {}
    for N, I, Rs in rho_table.QUICK:
        for R in Rs:
            t1, t2, r = rho_table.rho(N, I, R)
            out[(N, I, R)] = r
            print(f"  N={N} I={I} R={R}: {t1:.3g} s / {t2:.3g} s per sweep, rho {r:.1f}", flush=True)
    assert all(r > 1.0 for r in out.values()), out
    assert out[(7, 7, 10)] > out[(5, 14, 10)] > 1.5, out
