"""GPU parity: libxyz against the CPU oracle on the same seeded inputs.

+-1 data: pair sets, every pair statistic (s, stat, first_rep, hits) and every
per-repetition statistic (candidates, passed, fresh, cmask, max_bucket) must be
bit-identical.  Real data: the same pair set and values within 1e-12 relative
of the binary64 oracle (both sides decide membership in binary64; only pairs
whose value lies within that rounding band of kappa may differ).
"""
import sys

import numpy as np
import pytest

import oracle
import synthgen
import paper_1610_05108_amd as xyz

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


def assert_same_binary(res, ref_pairs, ref_reps):
    got = res["pairs"]
    assert len(got) == len(ref_pairs), (len(got), len(ref_pairs))
    for f in ("j", "k", "s", "first_rep", "hits"):
        assert np.array_equal(got[f], ref_pairs[f]), f
    assert np.array_equal(got["stat"], ref_pairs["stat"])
    reps = res["reps"]
    assert len(reps) == len(ref_reps)
    for f in ("candidates", "passed", "fresh", "cmask", "max_bucket"):
        assert np.array_equal(reps[f], ref_reps[f]), f


def run_both(ctx, XT, Y, m, L, kappa, seed=0, two_sided=False, rep_offset=0, rows=None, n=None, x=None):
    xh = x if x is not None else ctx.x_create(XT if n is None else synthgen.pack_bits_colmajor(XT), n=n)
    _log(f"case n={XT.shape[1]} p={XT.shape[0]} m={m} L={L} kappa={kappa} seed={seed} two={two_sided}")
    res = ctx.search(xh, Y, m=m, L=L, kappa=kappa, seed=seed, two_sided=two_sided, rep_offset=rep_offset, rows=rows)
    ref_pairs, ref_reps = oracle.search(XT, Y, m, L, kappa, seed=seed, two_sided=two_sided,
                                        rep_offset=rep_offset, rows=rows)
    return res, ref_pairs, ref_reps


def test_config1_bit_exact(ctx):
    d = synthgen.config1()
    p = d.params
    res, rp, rr = run_both(ctx, d.XT, d.Y, p["m"], p["L"], p["kappa"], seed=p["seed"])
    assert_same_binary(res, rp, rr)
    assert res["reps"]["candidates"].mean() > 1000


CASES = [
    # n, p, m, L, kappa, two_sided, seed
    (37, 33, 3, 7, 0.1, False, 1),
    (64, 64, 4, 5, -2.0, False, 2),
    (100, 257, 5, 9, 0.2, True, 3),
    (1000, 3000, 7, 6, 0.12, False, 4),
    (1025, 1500, 9, 4, -2.0, False, 5),     # every candidate survives: large merge
    (4097, 700, 6, 5, 0.05, True, 6),
    (33, 2, 1, 3, -2.0, False, 7),
    (200, 1, 2, 3, 0.0, False, 8),
    (500, 2000, 15, 30, 0.1, False, 9),
    (300, 800, 0, 2, 0.15, False, 10),       # m = 0: every pair collides
    (300, 800, 0, 2, 0.15, True, 11),
]


@pytest.mark.parametrize("n,p,m,L,kappa,two,seed", CASES)
def test_random_binary_bit_exact(ctx, n, p, m, L, kappa, two, seed):
    d = synthgen.small_binary(n, p, seed=seed, y_bias=0.4 + 0.05 * (seed % 3))
    res, rp, rr = run_both(ctx, d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two)
    assert_same_binary(res, rp, rr)


def test_packed_bits_input(ctx):
    d = synthgen.small_binary(130, 400, seed=12)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 5, 6, 0.1, seed=3, n=130)
    assert_same_binary(res, rp, rr)


def test_genotype_skewed_buckets(ctx):
    """Genotype-shaped columns give a few buckets far larger than the mean,
    so bucket products are split into many tiles."""
    XT, _ = synthgen.genotype(600, 5000, seed=13)
    r = np.random.default_rng(1)
    Y = np.where(r.random(600) < 0.45, 1, -1).astype(np.int8)
    res, rp, rr = run_both(ctx, XT, Y, 10, 6, 0.15, seed=2)
    assert_same_binary(res, rp, rr)
    assert res["reps"]["max_bucket"].max() > 8 * 5000 / 1024


def test_rows_table(ctx):
    d = synthgen.small_binary(150, 600, seed=14, planted=[(3, 9)], flip=0.2)
    rows = synthgen.rows_table(150, 8, 6, seed=5)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 6, 8, 0.2, rows=rows)
    assert_same_binary(res, rp, rr)


def test_survivor_buffer_growth(ctx):
    """More survivors than the initial buffer: the library grows it and redoes the chunk."""
    d = synthgen.small_binary(64, 2600, seed=15)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 3, 2, -2.0, seed=1)
    assert len(rp) > 1 << 17
    assert_same_binary(res, rp, rr)


def test_tile_list_growth():
    """More tiles in a chunk than the initial tile list of a fresh context holds: the
    verification kernels see the overflow on the device and verify nothing, the library
    grows the list and redoes the chunk; a second search reuses the grown list."""
    d = synthgen.small_binary(64, 40000, seed=41, planted=[(1, 39998)], flip=0.05)
    rp, rr = oracle.search(d.XT, d.Y, 12, 80, 0.5, seed=41)
    c = xyz.Context(0)
    try:
        x = c.x_create(d.XT)
        for it in range(2):
            _log(f"tile list growth: search {it}")
            res = c.search(x, d.Y, m=12, L=80, kappa=0.5, seed=41)
            assert res["timing"]["tiles"] > 1 << 16
            assert_same_binary(res, rp, rr)
    finally:
        c.close()


def test_one_host_wait_per_chunk():
    """The LDS bucket path waits on the stream once per chunk of repetitions
    (survivor count and tile-list sizes in one transfer), plus once after the
    inputs are checked and twice for the merged result; the sort path (m > 15)
    three times per chunk.  L = 4500 spans two chunks of at most 4096."""
    d = synthgen.small_binary(64, 1500, seed=42, planted=[(3, 1400)], flip=0.05)
    c = xyz.Context(0)
    try:
        x = c.x_create(d.XT)
        for m, per_chunk in ((8, 1), (16, 3)):
            for it in range(2):          # the first search may grow its workspaces and redo a chunk
                res = c.search(x, d.Y, m=m, L=4500, kappa=0.5, seed=3)
            t = res["timing"]
            _log(f"m={m}: chunks {t['chunks']}, host waits {t['host_syncs']}")
            assert t["chunks"] == 2
            assert t["host_syncs"] == per_chunk * t["chunks"] + 3
        small = c.search(x, d.Y, m=6, L=5, kappa=0.5, seed=3)
        assert small["timing"]["chunks"] == 1 and small["timing"]["host_syncs"] <= 5
    finally:
        c.close()


def test_split_repetitions_match_full_run(ctx):
    d = synthgen.small_binary(300, 1200, seed=16, planted=[(1, 2)], flip=0.1)
    x = ctx.x_create(d.XT)
    full = ctx.search(x, d.Y, m=6, L=10, kappa=0.12, seed=9)
    a = ctx.search(x, d.Y, m=6, L=4, kappa=0.12, seed=9, rep_offset=0)
    b = ctx.search(x, d.Y, m=6, L=6, kappa=0.12, seed=9, rep_offset=4)
    for f in ("candidates", "passed", "cmask", "max_bucket"):
        assert np.array_equal(full["reps"][f], np.concatenate([a["reps"][f], b["reps"][f]]))
    merged = {}
    for part in (a, b):
        for rec in part["pairs"]:
            key = (int(rec["j"]), int(rec["k"]))
            h, f = merged.get(key, (0, 1 << 30))
            merged[key] = (h + int(rec["hits"]), min(f, int(rec["first_rep"])))
    assert merged == {(int(r["j"]), int(r["k"])): (int(r["hits"]), int(r["first_rep"])) for r in full["pairs"]}


def test_batch_matches_single_searches(ctx):
    """Several responses against one X share projections and bucket sort; each
    result must equal its stand-alone search (and the oracle)."""
    XT = synthgen.rademacher(400, 1500, seed=17)
    r = np.random.default_rng(3)
    Ys = [np.where(r.random(400) < 0.5, 1, -1).astype(np.int8) for _ in range(5)]
    x = ctx.x_create(XT)
    params = [dict(m=7, L=6, kappa=0.1 + 0.01 * q, seed=4) for q in range(5)]
    params[3] = dict(m=5, L=6, kappa=0.1, seed=4)            # a different group
    params[4] = dict(m=7, L=6, kappa=0.1, seed=4, two_sided=True)
    batch = ctx.search_batch(x, Ys, params)
    for q in range(5):
        kw = params[q]
        single = ctx.search(x, Ys[q], **kw)
        assert np.array_equal(batch[q]["pairs"], single["pairs"]), q
        assert np.array_equal(batch[q]["reps"], single["reps"]), q
        rp, rr = oracle.search(XT, Ys[q], kw["m"], kw["L"], kw["kappa"], seed=kw["seed"],
                               two_sided=kw.get("two_sided", False))
        assert_same_binary(batch[q], rp, rr)


def test_device_tensor_inputs(ctx):
    torch = pytest.importorskip("torch")
    d = synthgen.small_binary(257, 900, seed=18, planted=[(5, 6)], flip=0.15)
    XT_d = torch.from_numpy(d.XT).cuda()
    Y_d = torch.from_numpy(d.Y).cuda()
    x = ctx.x_create(XT_d)
    res = ctx.search(x, Y_d, m=6, L=5, kappa=0.15, seed=2)
    rp, rr = oracle.search(d.XT, d.Y, 6, 5, 0.15, seed=2)
    assert_same_binary(res, rp, rr)


def assert_same_real(res, rp, rr, kappa, n, tol=1e-12):
    got = res["pairs"]
    gk = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(got["j"], got["k"]))}
    rk = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(rp["j"], rp["k"]))}
    for key in set(gk) ^ set(rk):
        src = got[gk[key]] if key in gk else rp[rk[key]]
        assert abs(src["value"] / n - kappa) <= tol * (1 + abs(src["value"]) / n), key
    for key in set(gk) & set(rk):
        g, r = got[gk[key]], rp[rk[key]]
        assert abs(g["value"] - r["value"]) <= tol * max(1.0, abs(r["value"])) * n
        assert g["hits"] == r["hits"] and g["first_rep"] == r["first_rep"]
    for f in ("candidates", "cmask", "max_bucket"):
        assert np.array_equal(res["reps"][f], rr[f]), f


@pytest.mark.parametrize("n,p,m,L,kappa,two,seed", [
    (300, 400, 6, 8, 0.2, False, 1),
    (1000, 1200, 8, 5, 0.3, False, 2),
    (97, 150, 3, 6, -1e300, False, 3),
    (513, 600, 7, 4, 0.25, True, 4),
])
def test_continuous_x_and_y(ctx, n, p, m, L, kappa, two, seed):
    d = synthgen.small_continuous(n, p, seed=seed, planted=[(0, 1), (7, 40)], noise=0.8)
    x = ctx.x_create(d.XT)
    _log(f"continuous n={n} p={p} m={m} L={L}")
    res = ctx.search(x, d.Y, m=m, L=L, kappa=kappa, seed=seed, two_sided=two)
    rp, rr = oracle.search(d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two)
    assert_same_real(res, rp, rr, kappa, n)


@pytest.mark.parametrize("ydtype", [np.float32, np.float64])
def test_binary_x_real_y(ctx, ydtype):
    d = synthgen.small_binary(400, 900, seed=19)
    r = np.random.default_rng(7)
    Y = (d.XT[2].astype(np.float64) * d.XT[11] + r.standard_normal(400)).astype(ydtype)
    Y[::17] = 0.0
    x = ctx.x_create(d.XT)
    res = ctx.search(x, Y, m=6, L=7, kappa=0.2, seed=5)
    rp, rr = oracle.search(d.XT, Y, 6, 7, 0.2, seed=5)
    assert_same_real(res, rp, rr, 0.2, 400)


def test_real_x_binary_y(ctx):
    d = synthgen.small_continuous(350, 500, seed=20)
    Y = np.where(np.random.default_rng(2).random(350) < 0.5, 1, -1).astype(np.int8)
    x = ctx.x_create(d.XT)
    res = ctx.search(x, Y, m=5, L=6, kappa=0.15, seed=1)
    rp, rr = oracle.search(d.XT, Y, 5, 6, 0.15, seed=1)
    assert_same_real(res, rp, rr, 0.15, 350)


def test_invalid_inputs_raise(ctx):
    d = synthgen.small_binary(40, 20, seed=21)
    x = ctx.x_create(d.XT)
    Y = d.Y.copy()
    Y[5] = 0
    with pytest.raises(xyz.XyzError) as e:
        ctx.search(x, Y, m=2, L=2, kappa=0.1)
    assert e.value.code == xyz.XYZ_EINVAL
    bad = d.XT.copy()
    bad[3, 4] = 3
    with pytest.raises(xyz.XyzError):
        ctx.x_create(bad)
    with pytest.raises(xyz.XyzError):
        ctx.search(x, d.Y, m=31, L=2, kappa=0.1)
    with pytest.raises(xyz.XyzError):
        ctx.search(x, d.Y, m=2, L=0, kappa=0.1)
    with pytest.raises(xyz.XyzError):
        ctx.search(x, d.Y, m=2, L=2, kappa=float("nan"))
    with pytest.raises(xyz.XyzError):
        ctx.search(x, np.zeros(40, dtype=np.float32), m=2, L=2, kappa=0.1)
    # the context stays usable after rejected calls
    res = ctx.search(x, d.Y, m=2, L=2, kappa=0.1)
    rp, rr = oracle.search(d.XT, d.Y, 2, 2, 0.1)
    assert_same_binary(res, rp, rr)


# ------------------------------------------------------------- brute force --

def _brute_ref(XT, Y, kappa, colsA=None, colsB=None, two_sided=False):
    """Expected exact result over colsA x colsB from the oracle's brute force."""
    p = XT.shape[0]
    full = oracle.brute(XT, Y, -2.0)
    val = {(int(r["j"]), int(r["k"])): int(r["s"]) for r in full}
    A = range(p) if colsA is None else colsA
    B = range(p) if colsB is None else colsB
    n = XT.shape[1]
    keep = set()
    for a in A:
        for b in B:
            if a == b:
                continue
            key = (min(a, b), max(a, b))
            sv = val[key]
            st = sv / n
            if (abs(st) > kappa) if two_sided else (st > kappa):
                keep.add(key)
    return {k: val[k] for k in keep}


@pytest.mark.parametrize("n,p,kappa,two,seed", [
    (77, 300, 0.1, False, 1),
    (1000, 700, 0.08, False, 2),
    (4097, 520, 0.03, True, 3),
    (32, 257, 0.2, False, 4),
    (2000, 256, 0.0, False, 5),
    (64, 2400, 0.25, False, 6),       # 55 block pairs: grid not a multiple of 8
    (150, 3100, 0.3, True, 7),
])
def test_bruteforce_all_pairs_exact(ctx, n, p, kappa, two, seed):
    d = synthgen.small_binary(n, p, seed=seed, planted=[(1, 2)], flip=0.3)
    x = ctx.x_create(d.XT)
    _log(f"brute n={n} p={p} kappa={kappa} two={two}")
    res = ctx.bruteforce(x, d.Y, kappa, two_sided=two)
    ref = oracle.brute(d.XT, d.Y, kappa, two_sided=two)
    got = res["pairs"]
    assert len(got) == len(ref)
    for f in ("j", "k", "s", "stat"):
        assert np.array_equal(got[f], ref[f]), f
    assert np.all(got["first_rep"] == -1) and np.all(got["hits"] == 0)


def test_bruteforce_column_lists(ctx):
    d = synthgen.small_binary(300, 400, seed=6)
    x = ctx.x_create(d.XT)
    r = np.random.default_rng(0)
    A = r.choice(400, size=90, replace=False).astype(np.int32)
    B = np.concatenate([A[:20], r.choice(400, size=300, replace=True)]).astype(np.int32)  # overlap + repeats
    res = ctx.bruteforce(x, d.Y, 0.05, colsA=A, colsB=B)
    want = _brute_ref(d.XT, d.Y, 0.05, list(A), list(B))
    got = {(int(a), int(b)): int(s) for a, b, s in zip(res["pairs"]["j"], res["pairs"]["k"], res["pairs"]["s"])}
    assert got == want
    assert list(zip(res["pairs"]["j"], res["pairs"]["k"])) == sorted(got)


def test_bruteforce_many_survivors(ctx):
    d = synthgen.small_binary(100, 600, seed=7)
    x = ctx.x_create(d.XT)
    res = ctx.bruteforce(x, d.Y, -2.0)
    ref = oracle.brute(d.XT, d.Y, -2.0)
    assert len(ref) == 600 * 599 // 2
    assert np.array_equal(res["pairs"]["s"], ref["s"]) and np.array_equal(res["pairs"]["j"], ref["j"])


def test_bruteforce_equals_exhaustive_search(ctx):
    """The matrix-core brute force and the popcount search with m = 0 compute
    the same set (two independent GPU routes to eq. (1))."""
    XT, _ = synthgen.genotype(2000, 3000, seed=8)
    Y = np.where(np.random.default_rng(5).random(2000) < 0.45, 1, -1).astype(np.int8)
    x = ctx.x_create(XT)
    b = ctx.bruteforce(x, Y, 0.06)
    s = ctx.search(x, Y, m=0, L=1, kappa=0.06)
    assert np.array_equal(b["pairs"][["j", "k", "s"]], s["pairs"][["j", "k", "s"]])
    assert len(b["pairs"]) > 100


def test_bruteforce_real_data(ctx):
    d = synthgen.small_continuous(200, 150, seed=9, planted=[(3, 4)])
    x = ctx.x_create(d.XT)
    res = ctx.bruteforce(x, d.Y, 0.2)
    ref = oracle.brute(d.XT, d.Y, 0.2)
    assert np.array_equal(res["pairs"][["j", "k"]], ref[["j", "k"]])
    assert np.allclose(res["pairs"]["value"], ref["value"], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("n,p,m,two,xbin", [
    (200, 300, 2, False, False),
    (100, 200, 1, False, False),
    (150, 400, 3, True, False),
    (190, 350, 2, False, True),
])
def test_real_large_buckets_matrix_tiles(ctx, n, p, m, two, xbin):
    """Buckets of 40-150 columns: products larger than one 32 x 32 tile on both
    sides are verified in 64 x 64 tiles on the FP64 matrix cores (every fragment
    count 1-4 per side, diagonal tiles of a bucket's own pairs, ragged edges)."""
    d = synthgen.small_continuous(n, p, seed=5, planted=[(0, 1)], noise=0.8)
    XT = d.XT
    if xbin:
        XT = np.where(d.XT < 0, -1, 1).astype(np.int8)
    x = ctx.x_create(XT)
    res = ctx.search(x, d.Y, m=m, L=2, kappa=0.05, seed=1, two_sided=two)
    rp, rr = oracle.search(XT, d.Y, m, 2, 0.05, seed=1, two_sided=two)
    assert_same_real(res, rp, rr, 0.05, n)
    assert len(rp) > 1000


@pytest.mark.parametrize("n,p,m,L,kappa,two,ybias,seed", [
    (1000, 2600, 5, 4, 0.12, False, 0.5, 41),   # ~81 columns per bucket: 64 + remainder tiles, all four fragment shapes
    (300, 3000, 6, 6, 0.2, True, 0.45, 42),     # ~47 per bucket: sides on both sides of 32, two-sided
    (129, 2900, 5, 3, 0.25, False, 1.0, 43),    # Y = +1: partner mask 0, diagonal tiles; one partial stage
    (5000, 2100, 5, 2, 0.05, False, 0.5, 44),   # 40 quads per column: many stages
])
def test_matrix_tile_fragment_shapes(ctx, n, p, m, L, kappa, two, ybias, seed):
    """Matrix-core tiles whose sides hold more or fewer than 32 columns (one or two
    fragment rows / columns per side), remainder tiles of buckets past 64 columns,
    and diagonal tiles of a bucket's own pairs, bit-exact against the oracle."""
    planted = [(0, 1), (5, 9)] if ybias < 1.0 else []      # planted pairs would drive Y
    d = synthgen.small_binary(n, p, seed=seed, planted=planted, flip=0.1, y_bias=ybias)
    res, rp, rr = run_both(ctx, d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two)
    assert rr["max_bucket"].max() > 64
    if ybias == 1.0:
        assert (rr["cmask"] == 0).all()
    assert_same_binary(res, rp, rr)


@pytest.mark.parametrize("n,p,ld_pad,device", [(200, 2000, 0, False), (77, 130, 5, False), (1025, 3001, 0, True),
                                               (64, 64, 64, True), (3, 1, 0, False)])
def test_rowmajor_int8_input_bit_exact(ctx, n, p, ld_pad, device):
    """X handed over as int8 +-1 in row-major order (XYZ_X_I8_PM1_ROWMAJOR), from
    host or device memory and with a leading dimension past p: the search equals
    the oracle bit for bit, and the exact search equals the one on the same X
    handed over column-major."""
    import ctypes
    import torch
    d = synthgen.small_binary(n, p, seed=n + p, planted=[(0, p - 1)] if p > 1 else [], flip=0.2)
    ld = p + ld_pad
    buf = np.ones((n, ld), dtype=np.int8)
    buf[:, :p] = d.XT.T
    _log(f"row-major case n={n} p={p} ld={ld} device={device}")
    if device:
        src = torch.from_numpy(buf).to("cuda:0")
        ptr, mem = src.data_ptr(), xyz.XYZ_MEM_DEVICE
    else:
        src = buf
        ptr, mem = buf.ctypes.data, xyz.XYZ_MEM_HOST
    h = ctypes.c_void_p()
    rc = xyz.lib().xyz_x_create(ctx.h, ptr, xyz.XYZ_X_I8_PM1_ROWMAJOR, mem, n, p, ld, None, ctypes.byref(h))
    assert rc == 0, xyz.lib().xyz_last_error()
    torch.cuda.synchronize()
    m, L, kappa = min(6, max(1, n // 20)), 9, 0.05
    res = ctx.search(h, d.Y, m=m, L=L, kappa=kappa, seed=3)
    rp, rr = oracle.search(d.XT, d.Y, m, L, kappa, seed=3)
    assert_same_binary(res, rp, rr)
    if p > 1:
        xc = ctx.x_create(d.XT)
        a = ctx.bruteforce(h, d.Y, -0.1)["pairs"]
        b = ctx.bruteforce(xc, d.Y, -0.1)["pairs"]
        assert len(a) == len(b) and all(np.array_equal(a[f], b[f]) for f in ("j", "k", "s"))
        ctx.x_destroy(xc)
    xyz.xyz_x_destroy(h)


def test_rowmajor_rejects_bad_values(ctx):
    X = np.ones((40, 70), dtype=np.int8)
    X[17, 33] = 0
    with pytest.raises(xyz.XyzError) as ei:
        ctx.x_create(X, row_major=True)
    assert ei.value.code == xyz.XYZ_EINVAL
    import ctypes
    h = ctypes.c_void_p()
    ok = np.ones((40, 70), dtype=np.int8)
    # leading dimension shorter than a row
    rc = xyz.lib().xyz_x_create(ctx.h, ok.ctypes.data, xyz.XYZ_X_I8_PM1_ROWMAJOR, xyz.XYZ_MEM_HOST, 40, 70, 69, None,
                                ctypes.byref(h))
    assert rc == xyz.XYZ_EINVAL
    x = ctx.x_create(ok, row_major=True)
    assert xyz.xyz_x_n(x) == 40 and xyz.xyz_x_p(x) == 70


def test_binding_checks_sizes_against_x(ctx):
    """The binding refuses responses and projection matrices whose length does not
    match n (the C side would read n entries), and weights that do not fit int32."""
    d = synthgen.small_binary(50, 30, seed=24)
    x = ctx.x_create(d.XT)
    with pytest.raises(ValueError):
        ctx.search(x, d.Y[:49], m=2, L=2, kappa=0.1)
    with pytest.raises(ValueError):
        ctx.bruteforce(x, np.concatenate([d.Y, d.Y]), 0.1)
    with pytest.raises(ValueError):
        ctx.dense_search(x, d.Y, np.zeros((2, 49), dtype=np.int32), 1, 0.1)
    wide = np.zeros((1, 50), dtype=np.int64)
    wide[0, 3] = 1 << 31
    with pytest.raises(ValueError):
        ctx.dense_search(x, d.Y, wide, 1, 0.1)
    ctx.search(x, d.Y, m=2, L=2, kappa=0.1)


BIG_CASES = [
    # n, p, m, L, kappa, two_sided, seed: bucket products past 64 x 96 columns (LDS-staged tiles)
    (1025, 3000, 2, 4, 0.08, False, 31),     # buckets of ~750: 3 x 3 block pairs, ragged last blocks
    (2000, 5000, 3, 3, 0.06, True, 32),      # two-sided: partners b ^ c and b ^ ~c
    (5000, 2100, 1, 3, 0.04, False, 33),     # n = 5000: five staged chunks of 1024 rows
    (700, 1100, 2, 3, -2.0, False, 34),      # every candidate survives: the pair-by-pair pass everywhere
    (333, 900, 0, 1, 0.1, False, 35),        # m = 0: one bucket, its own pairs as triangular block pairs
    (64, 600, 1, 6, 0.2, True, 36),          # one chunk of one quad
    (4097, 1300, 2, 2, 0.05, False, 37),     # a partial last chunk (33 quads)
    (700, 8400, 5, 2, 0.12, False, 38),      # buckets of ~262: thin remainders go to matrix-core strips
    (300, 2200, 3, 3, 0.1, True, 39),        # buckets of ~275, two-sided: strips on both sides
]


@pytest.mark.parametrize("n,p,m,L,kappa,two,seed", BIG_CASES)
def test_big_bucket_products_bit_exact(ctx, n, p, m, L, kappa, two, seed):
    d = synthgen.small_binary(n, p, seed=seed, planted=[(1, p - 2), (5, 17)], flip=0.3)
    res, rp, rr = run_both(ctx, d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two)
    assert_same_binary(res, rp, rr)
    assert res["reps"]["max_bucket"].max() > 96
