"""lyap_seed_apply_noalloc: the seed Lyapunov solve with a low-rank right-hand
side, with its work area in the library's fixed per-GPU array (no device
allocation), against lyap_seed_apply, which allocates its work area on the
seed.  Called through the C ABI; two calls in a row, the second with a smaller
batch (the area keeps the first call's contents), in both seed bases; a batch
beyond the area's capacity is an argument error."""
import ctypes as C

import numpy as np
import pytest

from gen import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as L
    L.load()
    return L, torch


def _call(lib, fn, seed, Y, G, torch):
    st = getattr(lib, fn)(seed.h, Y.shape[0], C.c_void_p(Y.data_ptr()), C.c_void_p(G.data_ptr()),
                          0, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("basis,maker", [
    ("eig", lambda: W.config(1, P=8)),                        # n = 2000, r = 2: several GEMM tiles
    ("eig", lambda: W.small_chain(45, (7, 30, 41), 4, 6)),    # ragged n = 90, r = 3
    ("schur", lambda: W.small_chain(70, (9, 40), 3, 4)),      # Schur basis, n = 140
])
def test_noalloc_matches_allocating_entry_point(basis, maker):
    L, torch = _lib()
    lib = L.load()
    pr = maker()
    seed = L.Seed.from_problem(pr, basis=basis)
    assert seed.info()["basis"] == (1 if basis == "eig" else 2)
    gen = torch.Generator(device="cpu").manual_seed(3)
    for batch in (7, 3):                # second call smaller: stale contents must not leak
        print("noalloc %s n=%d r=%d batch=%d" % (basis, pr.n, pr.r, batch), flush=True)
        Y = torch.randn((batch, pr.r, pr.n), generator=gen, dtype=torch.float64).cuda()
        G0 = torch.full_like(Y, float("nan"))
        G1 = torch.full_like(Y, float("nan"))
        assert _call(lib, "lyap_seed_apply", seed, Y, G0, torch) == 0
        assert _call(lib, "lyap_seed_apply_noalloc", seed, Y, G1, torch) == 0
        torch.cuda.synchronize()
        g0, g1 = G0.cpu().numpy(), G1.cpu().numpy()
        assert np.all(np.isfinite(g1))
        err = np.max(np.abs(g1 - g0)) / np.max(np.abs(g0))
        print("  max |diff| / max |G| = %.2e" % err, flush=True)
        assert err <= 1e-13
    seed.release()


def test_noalloc_rejects_a_batch_beyond_its_area():
    L, torch = _lib()
    lib = L.load()
    pr = W.config(1, P=8)                    # ld = 2048, r = 2: 229 KiB per batch entry
    seed = L.Seed.from_problem(pr)
    batch = 200                              # 45 MiB of work area > 32 MiB
    Y = torch.zeros((batch, pr.r, pr.n), dtype=torch.float64, device="cuda")
    G = torch.zeros_like(Y)
    assert _call(lib, "lyap_seed_apply_noalloc", seed, Y, G, torch) == 1   # LYAP_E_INVAL
    assert b"32" in lib.lyap_last_error() or b"work area" in lib.lyap_last_error()
    # a batch that fits still works afterwards
    Y = torch.ones((4, pr.r, pr.n), dtype=torch.float64, device="cuda")
    G0, G1 = torch.zeros_like(Y), torch.zeros_like(Y)
    assert _call(lib, "lyap_seed_apply", seed, Y, G0, torch) == 0
    assert _call(lib, "lyap_seed_apply_noalloc", seed, Y, G1, torch) == 0
    torch.cuda.synchronize()
    assert torch.allclose(G0, G1, rtol=1e-13, atol=0)
    seed.release()
