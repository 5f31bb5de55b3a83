"""Host-only checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments, and its block schedule equals the
oracle's bit for bit (integer work: exact)."""
import ctypes
import os
import re

import pytest

from oracle import schedule as osch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kpp():
    lib = os.path.join(ROOT, "paper_2501_11673_amd", "libkpp.so")
    if not os.path.exists(lib):
        import __graft_entry__

        __graft_entry__.build()
    import paper_2501_11673_amd as k

    return k


def header_symbols():
    text = open(os.path.join(ROOT, "include", "kpp.h")).read()
    return re.findall(r"KPP_API\s+[\w\s\*]+?\b(kpp_\w+)\s*\(", text)


def test_library_exports_every_declared_symbol(kpp):
    syms = header_symbols()
    assert len(syms) >= 10
    raw = ctypes.CDLL(kpp.LIB_PATH)
    for name in syms:
        assert hasattr(raw, name), name
    assert set(syms) == set(kpp.EXPORTED)
    assert kpp.kpp_abi_version() == 6


def test_params_default_and_validation(kpp):
    p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    assert p.lambda_ == 1e-8 and p.rho0 == 0.0 and p.eta < 0 and p.memo == kpp.KPP_MEMO_ONLINE
    assert p.accel == 1 and p.adaptive_rho == 1 and p.confirm_true_residual == 1
    with pytest.raises(kpp.KppError) as e:
        kpp.kpp_params_default(7)
    assert e.value.status == kpp.KPP_ERR_INVALID_ARG
    with pytest.raises(kpp.KppError):
        kpp.kpp_system_create(0, 0, 10, 10, 0, 10, 0)
    # schedule generator rejects s > rows
    p.block_size = 11
    with pytest.raises(kpp.KppError):
        kpp.kpp_schedule_generate(kpp.KPP_CD_PSD, 10, 10, p, 5, 100)


@pytest.mark.parametrize("seed,N", [(0, 1), (9, 4096), (0x2501116730, 1000), (2 ** 64 - 1, 77)])
def test_rht_signs_match_oracle(kpp, seed, N):
    from oracle import rht as orht

    assert kpp.kpp_rht_signs(seed, N) == [int(v) for v in orht.rademacher(seed, N)]


def test_rht_argument_checks(kpp):
    with pytest.raises(kpp.KppError) as e:
        kpp.kpp_rht_general(0, 4, 4, 0, 4, 0, 0, 4, 0, 4, 0)
    assert e.value.status == kpp.KPP_ERR_INVALID_ARG
    with pytest.raises(kpp.KppError):
        kpp.kpp_rht_psd(0, 4, 0, 4, 0, 0, 4, 0, 4, 0)
    with pytest.raises(kpp.KppError):
        kpp.kpp_rht_vector(0, 4, 0, 0, 4, 0, 0)
    with pytest.raises(kpp.KppError):
        kpp.kpp_rht_signs(1, -1)
    p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
    # several right-hand sides: a NULL system (or B, X) is refused before any device work
    for sys_, B, X in ((0, 8, 8), (8, 0, 8), (8, 8, 0)):
        with pytest.raises(kpp.KppError) as e:
            kpp.kpp_solve_multi(sys_, p, 2, B, 2, X, 2)
        assert e.value.status == kpp.KPP_ERR_INVALID_ARG
    assert p.rht == 0 and p.rht_seed == 0
    assert p.projection == kpp.KPP_PROJ_EXACT and p.lsqr_iters == 8 and p.sketch_size == 0


def oracle_schedule(kind, m, n, mode, s, T, seed, num_blocks=0, partition=True):
    N = n if kind == "psd" else m
    return osch.make_schedule(mode, N, s, T, seed, B0=osch.online_rate(kind, m, n, s),
                              num_blocks=num_blocks, partition=partition)


CASES = [
    ("general", 1000, 200, "online", 20, 3000, 101, 0, True),
    ("general", 2048, 32768, "online", 128, 600, 404, 0, True),
    ("general", 300, 5000, "online", 64, 900, 414, 0, True),
    ("psd", 4096, 4096, "online", 128, 2500, 202, 0, True),
    ("psd", 1000, 1000, "fixed", 128, 500, 212, 0, True),
    ("general", 6000, 700, "fixed", 256, 500, 313, 0, True),
    ("general", 500, 40, "fixed", 7, 400, 9, 33, False),
    ("psd", 97, 97, "off", 5, 120, 3, 0, True),
    ("psd", 1, 1, "fixed", 1, 10, 1, 0, True),
    # row counts on both sides of the library's bitmap ordering of a subset
    # (up to 2^18 rows) and a partition far above it
    ("general", 262144, 64, "online", 128, 120, 79, 0, True),
    ("general", 300000, 64, "online", 64, 200, 77, 0, True),
    ("general", 300000, 64, "fixed", 256, 100, 78, 0, True),
]


@pytest.mark.parametrize("kind,m,n,mode,s,T,seed,nb,part", CASES)
def test_schedule_matches_oracle_exactly(kpp, kind, m, n, mode, s, T, seed, nb, part):
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    p = kpp.kpp_params_default(ck)
    p.block_size = s
    p.seed = seed
    p.memo = {"online": kpp.KPP_MEMO_ONLINE, "fixed": kpp.KPP_MEMO_FIXED, "off": kpp.KPP_MEMO_OFF}[mode]
    p.num_blocks = nb
    p.fixed_partition = 1 if part else 0
    ref = oracle_schedule(kind, m, n, mode, s, T, seed, nb, part)
    steps, rows, lens = kpp.kpp_schedule_generate(ck, m, n, p, T, len(ref.blocks) + 8)
    assert steps == ref.step_block.tolist()
    assert len(rows) == len(ref.blocks)
    for b, blk in enumerate(ref.blocks):
        assert lens[b] == len(blk)
        assert rows[b][:lens[b]] == blk.tolist()
        assert all(v == -1 for v in rows[b][lens[b]:])


def test_schedule_rejects_small_capacity(kpp):
    p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    p.block_size = 10
    p.memo = kpp.KPP_MEMO_FIXED
    with pytest.raises(kpp.KppError):
        kpp.kpp_schedule_generate(kpp.KPP_CD_PSD, 100, 100, p, 5, 3)


def test_explicit_schedule_is_used_as_given(kpp):
    """A caller-given schedule replaces the generator: the steps come back as
    given and the table as given (padding -1)."""
    p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
    p.block_size = 4
    table = [[0, 3, 7, 9], [1, 2, -1, -1], [4, 5, 6, 8]]
    steps = [2, 0, 0, 1, 2, 1, 0]
    keep = kpp.kpp_set_schedule(p, steps, table)
    got_steps, rows, lens = kpp.kpp_schedule_generate(kpp.KPP_KACZMARZ, 10, 6, p, len(steps), 3)
    assert got_steps == steps
    assert rows == table and lens == [4, 2, 4]
    with pytest.raises(kpp.KppError):
        kpp.kpp_schedule_generate(kpp.KPP_KACZMARZ, 10, 6, p, len(steps) + 1, 3)
    del keep


@pytest.mark.parametrize("table,steps", [
    ([[0, 3, 2, 9]], [0]),            # rows not ascending
    ([[0, 3, 7, 10]], [0]),           # row out of range (10 rows)
    ([[0, -1, 7, 9]], [0]),           # a row after the padding
    ([[-1, -1, -1, -1]], [0]),        # empty block
    ([[0, 1, 2, 3]], [0, 1]),         # block id out of range
])
def test_explicit_schedule_rejects_malformed_input(kpp, table, steps):
    p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
    p.block_size = 4
    keep = kpp.kpp_set_schedule(p, steps, table)
    with pytest.raises(kpp.KppError):
        kpp.kpp_schedule_generate(kpp.KPP_KACZMARZ, 10, 6, p, len(steps), 4)
    del keep
