"""CPU-side checks of the C-ABI library: it loads and exports every declared symbol."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lyapsmw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary_entry_points():
    syms = declared_symbols()
    for s in ("seed_factor", "lyap_seed_apply", "smw_solve_batch", "trace_EX"):
        assert s in syms


def test_library_loads_and_exports_every_declared_symbol():
    import paper_2312_08201_amd as L
    path = L.lyapsmw.LIB_PATH if hasattr(L, "lyapsmw") else None
    lib = L.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(L.EXPORTS) == set(declared_symbols())


def test_status_strings_without_gpu():
    import paper_2312_08201_amd as L
    lib = L.load()
    assert lib.lyap_status_string(0) == b"ok"
    assert lib.lyap_status_string(3) == b"unstable or singular seed"


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_2312_08201_amd as L
    from gen import workloads as W
    pr = W.small_chain(10, (3,), 2, 2)
    with pytest.raises(RuntimeError):
        L.Seed.from_problem(pr)


@pytest.mark.parametrize("n,seed", [(7, 0), (40, 1), (150, 2)])
def test_host_real_schur_matches_definition(n, seed):
    """The library's Francis QR: A = Z T Z^T, Z orthogonal, standard quasi-triangular T,
    eigenvalues equal to LAPACK's."""
    import numpy as np
    import paper_2312_08201_amd as L
    from gen import workloads as W
    A = W.random_stable(n, 1, 1, 1, seed).A0
    T, Z = L.real_schur(A)
    assert np.linalg.norm(Z @ T @ Z.T - A) <= 1e-13 * np.linalg.norm(A)
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 1e-13 * n
    assert np.all(np.tril(T, -2) == 0)
    for i in range(n - 1):
        if T[i + 1, i] != 0:  # 2x2 block: complex pair, not followed by another subdiagonal
            assert i + 2 >= n or T[i + 2, i + 1] == 0
            a, b, c, d = T[i, i], T[i, i + 1], T[i + 1, i], T[i + 1, i + 1]
            assert (0.5 * (a - d)) ** 2 + b * c < 0
    ev = np.linalg.eigvals(T)
    ref = np.linalg.eigvals(A)
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert np.allclose(sorted(ev, key=key), sorted(ref, key=key), atol=1e-10)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
