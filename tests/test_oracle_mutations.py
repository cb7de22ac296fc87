"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch each one: a flipped adjoint sign, the other reading of the prox
weight, a dropped extrapolation factor, a component-wise flux shrink and a
dropped boundary term of D."""
import numpy as np
import pytest

from oracle import ops, uot
from tests import test_oracle_ops as T_ops
from tests import test_oracle_pins as T_pins


def _fails(fn, *a, **k):
    try:
        fn(*a, **k)
    except AssertionError:
        return True
    return False


def test_pins_pass_unmutated():
    assert not _fails(T_pins.test_1d_balanced_is_cumsum, 9)
    assert not _fails(T_ops.test_projection_update_vs_brute_force, 1)


def test_flipped_adjoint_sign_is_caught(monkeypatch):
    orig = ops.div_adj
    monkeypatch.setattr(ops, "div_adj", lambda a, bc=0: tuple(-g for g in orig(a, bc)))
    assert _fails(T_ops.test_adjoint_identity, (5, 7), 0)


def test_other_rho_reading_is_caught(monkeypatch):
    orig_iter = uot.iterate

    def wrong(prob, st, tau1, tau2):
        # theta = rho tau1 / (1 + rho tau1) with rho taken as the prox step
        rho = prob.rho
        eff = 1.0 / rho  # makes tau1/(eff + tau1) equal the other reading
        return orig_iter(uot.with_(prob, rho=eff), st, tau1, tau2)
    monkeypatch.setattr(uot, "iterate", wrong)
    assert _fails(T_ops.test_projection_update_vs_brute_force, 1)


def test_dropped_extrapolation_is_caught(monkeypatch):
    def no_extrap(prob, st, tau1, tau2):
        gx, gy = ops.div_adj(st.a, prob.bc)
        Mx, My = ops.prox_flux(st.Mx - tau1 * gx, st.My - tau1 * gy, tau1, prob.norm)
        r = ops.shrink1(st.r + tau1 * st.a, prob.mu * tau1) if not prob.balanced else st.r
        k_new = uot.constraint(prob, Mx, My, st.x0, st.x1, r)
        return uot.State(Mx, My, r, st.a + tau2 * k_new, st.x0, st.x1)
    monkeypatch.setattr(uot, "iterate", no_extrap)
    assert _fails(T_ops.test_dual_update_extrapolation, 0, False)


def test_componentwise_shrink_is_caught(monkeypatch):
    monkeypatch.setattr(ops, "shrink2", lambda vx, vy, s: (ops.shrink1(vx, s), ops.shrink1(vy, s)))
    assert _fails(T_ops.test_group_shrink_vs_brute_force)


def test_dropped_boundary_term_is_caught(monkeypatch):
    orig = ops.div

    def wrong(Mx, My, bc=0):
        out = orig(Mx, My, bc)
        out[:, 0] -= np.asarray(Mx, dtype=np.float64)[:, -1]  # periodic wrap instead of zero flux
        return out
    monkeypatch.setattr(ops, "div", wrong)
    assert _fails(T_ops.test_div_matches_loop_assembled_matrix, (5, 7), 1)
