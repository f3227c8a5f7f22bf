"""Pins of the stability oracle (oracle/stability.py) against closed forms.

The filter of the agent-importance sweep (Section 4) discards parameter
samples whose A(d) = A0 - U diag(d) V^T has an eigenvalue with Re >= 0.
"""
import numpy as np
import pytest

from gen import workloads as W
from oracle import stability as S


def test_scalar_update():
    """A0 = -a, U = V = 1: the one eigenvalue is -a - d."""
    a = 1.7
    for d in np.linspace(-4.0, 3.0, 29):
        expect = 1 if -a - d >= 0.0 else 0
        assert S.unstable_count(np.array([[-a]]), np.ones((1, 1)), np.ones((1, 1)), [d]) == expect
        assert S.rightmost_real_part(np.array([[-a]]), np.ones((1, 1)), np.ones((1, 1)), [d]) == \
            pytest.approx(-a - d, abs=1e-15)


def test_diagonal_seed_full_rank_update():
    """A0 = diag(a), U = V = I: eigenvalues a_i - d_i exactly."""
    rng = np.random.default_rng(3)
    a = -rng.uniform(0.5, 3.0, 7)
    for _ in range(20):
        d = rng.uniform(-4.0, 1.0, 7)
        assert S.unstable_count(np.diag(a), np.eye(7), np.eye(7), d) == int(np.sum(a - d >= 0))


def test_rotation_block():
    """[[-al, w], [-w, -al]] - delta I has the pair -al - delta +- i w: both
    eigenvalues cross together."""
    al, w = 0.3, 2.0
    A0 = np.array([[-al, w], [-w, -al]])
    for delta in (-1.0, -0.31, -0.29, 0.5):
        expect = 2 if -al - delta >= 0 else 0
        assert S.unstable_count(A0, np.eye(2), np.eye(2), [delta, delta]) == expect
        ev = np.sort_complex(S.eigenvalues(A0, np.eye(2), np.eye(2), [delta, delta]))
        assert np.allclose(ev, [-al - delta - 1j * w, -al - delta + 1j * w], atol=1e-14)


def test_agent_example_inertia_identity():
    """The agents' A0 is symmetric negative definite and agent k's update is
    e_k e_k^T kron M(v), M = [[v1, v2], [v2, v3]].  Along -A0 + t Us M Us^T,
    t in [0, 1], definiteness is lost exactly when det(I + t M W) = 0 with
    W = Us^T (-A0)^-1 Us, i.e. when an eigenvalue of W^1/2 M W^1/2 is <= -1.
    That independent 2x2 test must agree with the rightmost eigenvalue."""
    A0 = W.agent_network(12, seed=5)
    D = W.agent_grid(step=2.0)
    for k in (0, 5, 11):
        Us = np.zeros((A0.shape[0], 2))
        Us[2 * k:2 * k + 2] = np.eye(2)
        Wm = Us.T @ np.linalg.solve(-A0, Us)
        ew, ev = np.linalg.eigh(Wm)
        Wh = ev @ np.diag(np.sqrt(ew)) @ ev.T
        pr = W.agent_problem(A0, k, D)
        cnt, rm = S.sweep(pr.A0, pr.U, pr.V, pr.d)
        checked = 0
        for i, d in enumerate(pr.d):
            if abs(rm[i]) < 1e-9:
                continue
            M = np.array([[d[0], d[1]], [d[2], d[3]]])
            mu = np.linalg.eigvalsh(Wh @ M @ Wh)
            assert (cnt[i] > 0) == bool(np.min(mu) <= -1.0), (k, d)
            checked += 1
        assert checked > 0.9 * pr.P
        assert 0 < np.mean(cnt > 0) < 1   # both kinds occur


def test_planted_sign_error_is_caught():
    """An oracle that adds the update instead of subtracting it fails the
    scalar pin."""
    def wrong(A0, U, V, d):
        return int(np.sum(np.linalg.eigvals(A0 + (U * np.asarray(d)[None, :]) @ V.T).real >= 0))
    a = 1.7
    bad = [d for d in np.linspace(-4.0, 3.0, 29)
           if wrong(np.array([[-a]]), np.ones((1, 1)), np.ones((1, 1)), [d]) != (1 if -a - d >= 0 else 0)]
    assert bad
