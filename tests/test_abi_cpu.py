"""Host-side checks of the C ABI (no GPU calls): the library loads, every
function declared in include/uot.h is exported, parameter validation
returns the documented codes, and the closed-form ||K||^2 agrees with the
oracle's."""
import os
import re

import pytest

from paper_1909_00149_amd import _lib
from paper_1909_00149_amd.uot import Params, check_params, knorm2, DIST, PROX, PROX_FIXED

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(uot\w*)\s*\(", text, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert "uot_solve" in names and "uot_solve_batched" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = _lib.load()
    for code in range(9):
        assert lib.uot_status_string(code)
    assert b"step" in lib.uot_status_string(_lib.UOT_ERR_STEP)


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(mode=3), _lib.UOT_ERR_ARG),
    (dict(residual_p=3), _lib.UOT_ERR_ARG),
    (dict(bc=2), _lib.UOT_ERR_ARG),
    (dict(mu=0.0), _lib.UOT_ERR_ARG),
    (dict(mu=0.0, balanced=True), 0),
    (dict(mode=PROX, rho=0.0), _lib.UOT_ERR_ARG),
    (dict(tau1=0.1, tau2=0.0), _lib.UOT_ERR_ARG),
    (dict(tau1=0.5, tau2=0.5), _lib.UOT_ERR_STEP),
    (dict(tau1=0.5, tau2=0.5, flags=_lib.UOT_UNSAFE_STEPS), 0),
    (dict(tau1=0.3, tau2=0.3), 0),
    (dict(max_iter=-1), _lib.UOT_ERR_ARG),
    (dict(tile_rows=5), _lib.UOT_ERR_ARG),
    (dict(tile_rows=16), 0),
    (dict(tile_rows=4016), 0),
    (dict(tile_rows=8032), 0),
    (dict(tile_rows=3016), _lib.UOT_ERR_ARG),
    (dict(tile_rows=4000), _lib.UOT_ERR_ARG),
    (dict(nx=10, ny=10, pitch=9), _lib.UOT_ERR_SHAPE),
    (dict(flags=_lib.UOT_ALLOW_SIGNED, mode=PROX), _lib.UOT_ERR_ARG),
    (dict(nx=-1), _lib.UOT_ERR_SHAPE),
    (dict(norm=1), 0),
    (dict(norm=1, bc=1, mode=PROX), 0),
    (dict(norm=2), _lib.UOT_ERR_ARG),
])
def test_check_params_codes(kw, code):
    base = dict(nx=16, ny=16, mu=1.0)
    base.update(kw)
    assert check_params(Params(**base)) == code


@pytest.mark.parametrize("mode", [DIST, PROX, PROX_FIXED])
@pytest.mark.parametrize("bal", [False, True])
@pytest.mark.parametrize("bc", [0, 1])
def test_knorm2_matches_oracle(mode, bal, bc):
    from oracle import ops
    for nx, ny in [(1, 1), (64, 64), (512, 37), (3, 1000)]:
        assert abs(knorm2(nx, ny, mode, bal, bc) - ops.knorm2(nx, ny, mode, bal, bc)) < 1e-12


@pytest.mark.parametrize("kw,ok", [({}, True), (dict(kappa=0.0), False), (dict(rho=-1.0), False),
                                   (dict(prox_iters=0), False), (dict(check_every=0), False),
                                   (dict(mu=0.0), False), (dict(mu=0.0, balanced=1), True),
                                   (dict(lam=-0.1), False), (dict(residual_p=3), False), (dict(nx=0), False),
                                   (dict(eps=float("nan")), False), (dict(prox_tau_ratio=0.01), True),
                                   (dict(prox_tau_ratio=-0.5), False),
                                   (dict(prox_tau_ratio=float("inf")), False)])
def test_uotdf_check_params(kw, ok):
    from paper_1909_00149_amd.admm import UotDf
    assert (UotDf.check(**kw) == 0) == ok


@pytest.mark.parametrize("kw,ok", [({}, True), (dict(frames=1), False), (dict(frames=65), False),
                                   (dict(frames=64), True), (dict(kappa=0.0), False), (dict(gam=-1.0), False),
                                   (dict(lam=0.0, gam=0.0), True), (dict(mu=0.0), False),
                                   (dict(mu=0.0, balanced=1), True), (dict(prox_iters=0), False),
                                   (dict(prox_tau_ratio=0.01), True), (dict(prox_tau_ratio=-1.0), False),
                                   (dict(signed_sparse=1), True), (dict(signed_sparse=2), False)])
def test_rpca_check_params(kw, ok):
    from paper_1909_00149_amd.admm import Rpca
    assert (Rpca.check(**kw) == 0) == ok


def test_library_matches_its_sources(monkeypatch):
    """The loader refuses a libuot.so whose recorded source digest is not
    the digest of the sources in the tree (a stale build)."""
    with open(_lib.DIGEST_PATH) as f:
        assert f.read().strip() == _lib.sources_digest()
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "sources_digest", lambda: "0" * 64)
    with pytest.raises(RuntimeError, match="not built from the current sources"):
        _lib.load()
