"""hlu_truncate_add_noalloc (static device scratch, no allocation) against
hlu_truncate_add (allocating): the same kernel on the same descriptors, so
ranks and factors must agree bit for bit; two calls in a row, the second
on a smaller update (the scratch keeps the first call's descriptors and must
be fully rewritten), each also within the Eckart-Young bound of the oracle's
truncation of the same sum."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def _case(torch, rng, m, n, kc, kx, cap):
    U0 = rng.standard_normal((m, kc)) * 0.6 ** np.arange(kc)
    V0 = rng.standard_normal((n, kc))
    X = rng.standard_normal((m, kx)) * 0.6 ** np.arange(kx) * 0.3
    Y = rng.standard_normal((n, kx))
    Ud = torch.zeros((cap, m), dtype=torch.float64, device="cuda")
    Vd = torch.zeros((cap, n), dtype=torch.float64, device="cuda")
    Ud[:kc] = torch.tensor(U0.T, device="cuda")
    Vd[:kc] = torch.tensor(V0.T, device="cuda")
    Xd = torch.tensor(X.T.copy(), device="cuda")
    Yd = torch.tensor(Y.T.copy(), device="cuda")
    return (U0, V0, X, Y), (Ud, Vd, Xd, Yd)


def test_noalloc_truncation_matches_allocating():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_00874_amd as P
    assert P.lib.hlu_static_scratch_bytes() == 4096
    rng = np.random.default_rng(2024)
    cap = 32
    for m, n, kc, kx, eps in [(300, 200, 16, 80, 1e-6), (40, 30, 5, 7, 1e-5)]:
        _say("noalloc truncation", m, n, kc, kx, eps)
        host, dev = _case(torch, rng, m, n, kc, kx, cap)
        dev2 = [t.clone() for t in dev]
        k_a = P.truncate_add(dev[0], dev[1], kc, dev[2], dev[3], cap, eps)
        k_s = P.truncate_add(dev2[0], dev2[1], kc, dev2[2], dev2[3], cap, eps, noalloc=True)
        torch.cuda.synchronize()
        assert k_a == k_s
        assert torch.equal(dev[0][:k_a], dev2[0][:k_s])
        assert torch.equal(dev[1][:k_a], dev2[1][:k_s])
        U0, V0, X, Y = host
        D = U0 @ V0.T - X @ Y.T
        Ug = dev2[0].cpu().numpy()[:k_s].T
        Vg = dev2[1].cpu().numpy()[:k_s].T
        sig = np.linalg.svd(D, compute_uv=False)
        k_o = O.Rule(eps=eps, cap=cap).choose(sig)
        err = np.linalg.norm(D - Ug @ Vg.T)
        _say("rank", k_s, "oracle rank", k_o, "error", err / np.linalg.norm(D))
        assert abs(k_s - k_o) <= 1
        assert err <= 1.01 * max(eps * np.linalg.norm(D), np.sqrt(np.sum(sig[k_s:] ** 2))) + 1e-13
