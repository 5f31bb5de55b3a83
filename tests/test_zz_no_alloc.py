"""The no-allocation block factor (kpp_block_factor_noalloc) against the
allocating one (kpp_block_factor) through the C ABI: two calls in a row, the
second with a smaller input, on Kaczmarz++ and CD++ systems; one block of each
call also against the oracle's regularized Gram and Cholesky factor
(Algorithm 1; Algorithm 2).

Bar: the factor data are floating point.  Where the Gram's column split is
the same on both paths the results are identical (checked bit for bit); where
the no-allocation path splits the columns into fewer chunks to fit its
scratch, the two differ only by the order of the Gram's sums, and the test
holds ||L_a - L_b|| / ||L_b|| <= 1e-10 (the spec bar for FP64 results)
on blocks whose Grams have condition numbers below 10 (Gaussian rows).
"""
import numpy as np
import pytest

from oracle import kpp as okpp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2501_11673_amd as kpp

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    ctx = kpp.kpp_context_create(0, torch.cuda.current_stream(dev).cuda_stream)
    yield kpp, torch, dev, ctx
    kpp.kpp_context_destroy(ctx)


def blocks(rng, N, s, nb, ragged):
    rows, lens = [], []
    for k in range(nb):
        ln = s if not ragged or k % 2 == 0 else max(1, s - 7 * (k + 1))
        r = np.sort(rng.choice(N, size=ln, replace=False)).astype(np.int32)
        rows.extend(list(r) + [0] * (s - ln))
        lens.append(ln)
    return rows, lens


def both(kpp, torch, dev, h, s, lam, rows, lens):
    nb = len(lens)
    La = torch.full((max(nb, 1) * s * s,), 7.0, dtype=torch.float64, device=dev)
    Lb = torch.full((max(nb, 1) * s * s,), -3.0, dtype=torch.float64, device=dev)
    kpp.kpp_block_factor(h, s, lam, rows, lens, La.data_ptr())
    kpp.kpp_block_factor_noalloc(h, s, lam, rows, lens, Lb.data_ptr())
    torch.cuda.synchronize()
    return La.cpu().numpy().reshape(-1, s, s), Lb.cpu().numpy().reshape(-1, s, s)


def check_oracle(A, kind, s, lam, rows, lens, Lnoalloc, k):
    ln = lens[k]
    S = np.asarray(rows[k * s:k * s + ln])
    G = okpp.regularized_gram(A, S, lam, kind)
    Lo = okpp.cholesky_lower(G)
    Lg = Lnoalloc[k].T[:ln, :ln]          # column-major slot -> row-major lower factor
    assert np.allclose(np.triu(Lnoalloc[k].T[:s, :s], 1), 0.0)
    err = np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo)
    assert err <= 1e-10, (kind, s, k, err)


# kind, (m, n), calls: [(s, nb, ragged)], the second call smaller than the first
CASES = [
    ("general", (3000, 2000), [(128, 6, False), (64, 2, True)]),
    ("general", (2048, 32768), [(128, 4, False), (100, 1, False)]),
    ("general", (1500, 700), [(300, 3, True), (256, 1, False)]),
    ("psd", (1000, 1000), [(100, 5, True), (40, 2, False)]),
    ("psd", (900, 900), [(300, 2, False), (129, 1, True)]),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1][0]}x{c[1][1]}" for c in CASES])
def test_noalloc_factor_matches_allocating_one(env, case):
    kpp, torch, dev, ctx = env
    kind, (m, n), calls = case
    rng = np.random.default_rng(2501 + m + n)
    if kind == "psd":
        X = rng.standard_normal((n, n + 50))
        A = X @ X.T / (n + 50) + 0.5 * np.eye(n)
        ck = kpp.KPP_CD_PSD
        N = n
    else:
        A = rng.standard_normal((m, n)) / np.sqrt(n)
        ck = kpp.KPP_KACZMARZ
        N = m
    b = rng.standard_normal(m)
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    h = kpp.kpp_system_create(ctx, ck, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        for s, nb, ragged in calls:
            print(f"[noalloc] {kind} {m}x{n} s={s} nb={nb} ragged={ragged}", flush=True)
            lam = 1e-6
            rows, lens = blocks(rng, N, s, nb, ragged)
            La, Lb = both(kpp, torch, dev, h, s, lam, rows, lens)
            same = np.array_equal(La, Lb)
            err = np.linalg.norm(La - Lb) / np.linalg.norm(La)
            print(f"[noalloc]   identical={same} rel diff {err:.3e}", flush=True)
            assert err <= 1e-10
            if kind == "psd":
                assert same   # CD++ Grams are a gather: no split to differ
            check_oracle(A, kind, s, lam, rows, lens, Lb, 0)
            check_oracle(A, kind, s, lam, rows, lens, Lb, nb - 1)
    finally:
        kpp.kpp_system_destroy(h)


def test_noalloc_identical_when_the_default_split_fits(env):
    """A Kaczmarz++ batch whose default split fits the scratch: bit for bit."""
    kpp, torch, dev, ctx = env
    rng = np.random.default_rng(77)
    m, n, s = 800, 1000, 64
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.zeros(m, dtype=torch.float64, device=dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        for nb in (3, 1):
            rows, lens = blocks(rng, m, s, nb, True)
            La, Lb = both(kpp, torch, dev, h, s, 1e-4, rows, lens)
            assert np.array_equal(La, Lb)
    finally:
        kpp.kpp_system_destroy(h)


def test_noalloc_rejects_oversized_staging(env):
    kpp, torch, dev, ctx = env
    m = n = 600
    A = torch.eye(n, dtype=torch.float64, device=dev)
    bd = torch.zeros(n, dtype=torch.float64, device=dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, m, n, A.data_ptr(), n, bd.data_ptr())
    try:
        s, nb = 512, 600          # nb * (s + 2) = 308400 > 262080 staged entries
        rows = [i % n for i in range(s)] * nb
        lens = [1] * nb
        L = torch.zeros(8, dtype=torch.float64, device=dev)
        with pytest.raises(kpp.KppError) as e:
            kpp.kpp_block_factor_noalloc(h, s, 1e-6, rows, lens, L.data_ptr())
        assert e.value.status == kpp.KPP_ERR_INVALID_ARG
        assert "no-allocation scratch" in str(e.value)
    finally:
        kpp.kpp_system_destroy(h)
