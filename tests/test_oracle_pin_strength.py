"""The oracle's pins catch plausible mistakes (CPU only).

Each mutant below is the oracle's definition with one planted mistake (a
dropped conjugate, a dropped mask, a wrong transform direction, a missing
centring shift, a transposed operand, an inverted CG ratio), built from the
oracle's own transform primitives.  Every mutant must fail at least one of
the pin checks that the real oracle passes (see test_oracle_operators.py and
test_oracle_cg.py).  Nothing here touches the GPU path.
"""
import numpy as np
import pytest

import oracle
from paper_1807_11830_amd import synth


def _E(x, S, m, fwd=-1, centred=True, transpose=False):
    Sx = np.swapaxes(S, -1, -2) if transpose else S
    out = []
    for c in range(S.shape[0]):
        u = Sx[c] * x
        k = oracle.centred_nd(u, fwd) if centred else np.fft.fft2(u, norm="ortho") if fwd < 0 else np.fft.ifft2(u, norm="ortho")
        out.append(k * m[:, None])
    return np.stack(out)


def _EH(y, S, m, inv=+1, conj=True, mask=True, centred=True, transpose=False):
    Sx = np.swapaxes(S, -1, -2) if transpose else S
    acc = 0
    for c in range(S.shape[0]):
        v = y[c] * (m[:, None] if mask else 1.0)
        img = oracle.centred_nd(v, inv) if centred else np.fft.ifft2(v, norm="ortho") if inv > 0 else np.fft.fft2(v, norm="ortho")
        acc = acc + (np.conj(Sx[c]) if conj else Sx[c]) * img
    return acc


MUTANTS = {
    "correct": ({}, {}),
    "no_conj": ({}, {"conj": False}),
    "no_mask_in_adjoint": ({}, {"mask": False}),
    "wrong_direction": ({"fwd": +1}, {"inv": -1}),
    "no_centring": ({"centred": False}, {"centred": False}),
    "transposed_maps": ({"transpose": True}, {"transpose": True}),
}


def _checks(Ef, EHf):
    """Return the failing pin names for an (E, E^H) pair."""
    fails = []
    n, nc = 8, 2
    rng = np.random.default_rng(0)
    S = rng.standard_normal((nc, n, n)) + 1j * rng.standard_normal((nc, n, n))
    m = synth.mask_regular(n, 2, 2)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((nc, n, n)) + 1j * rng.standard_normal((nc, n, n))
    lhs = np.vdot(Ef(x, S, m).ravel(), y.ravel())
    rhs = np.vdot(x.ravel(), EHf(y, S, m).ravel())
    if abs(lhs - rhs) > 1e-12 * abs(lhs):
        fails.append("adjoint")
    # Eq. (1) at full sampling (oracle-equivalent brute force definition)
    full = np.ones(n, np.uint8)
    ref = oracle.EH(y[None], S, full)[0]
    h = n // 2
    j = np.arange(n) - h
    K = np.exp(2j * np.pi * (np.outer(j, j) % n) / n)
    eq1 = sum(np.conj(S[i]) * (K @ y[i] @ K.T) / (n * n) for i in range(nc)) * np.sqrt(n * n)
    if np.linalg.norm(EHf(y, S, full) - eq1) > 1e-12 * np.linalg.norm(eq1):
        fails.append("eq1")
    assert np.linalg.norm(ref - eq1) <= 1e-12 * np.linalg.norm(eq1)
    return fails


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutants_fail_a_pin(name):
    ek, ehk = MUTANTS[name]
    fails = _checks(lambda x, S, m: _E(x, S, m, **ek), lambda y, S, m: _EH(y, S, m, **ehk))
    if name == "correct":
        assert fails == []
    else:
        assert fails, f"mutant {name} passed every pin"


def _cg_py(Ad, b, k, invert_beta=False, drop_alpha_in_r=False):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = np.vdot(r, r).real
    for _ in range(k):
        q = Ad @ p
        a = rho / np.vdot(p, q).real
        x = x + a * p
        r = r - (q if drop_alpha_in_r else a * q)
        rn = np.vdot(r, r).real
        beta = rho / rn if invert_beta else rn / rho
        p = r + beta * p
        rho = rn
    return x


@pytest.mark.parametrize("mut", ["invert_beta", "drop_alpha_in_r"])
def test_cg_mutants_fail_krylov_pin(mut):
    from test_oracle_cg import _dense_A, _krylov_minimiser, _tiny
    n, maps, mask, y = _tiny()
    Ad = _dense_A(n, maps, mask)
    b = oracle.EH(y, maps, mask).ravel()
    ref = _krylov_minimiser(Ad, b, 5)
    good = _cg_py(Ad, b, 5)
    assert np.linalg.norm(good - ref) <= 1e-9 * np.linalg.norm(ref)
    bad = _cg_py(Ad, b, 5, **{mut: True})
    assert np.linalg.norm(bad - ref) > 1e-6 * np.linalg.norm(ref)
