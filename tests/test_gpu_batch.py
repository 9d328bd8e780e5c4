"""Batched form: persistent tile-walking kernels in one HIP graph give the
same bits as the single-grid launches, on every replay, and match the
oracle."""
import numpy as np
import pytest
import torch

from paper_2303_12374_amd import inputs
from gpu_util import TOL, Case, outside_interior_mask, rel_err

pytestmark = pytest.mark.gpu


def kl():
    from paper_2303_12374_amd import kl as m
    return m


@pytest.fixture(autouse=True)
def no_wisdom(tmp_path):
    m = kl()
    m.kl_set_wisdom_dir(str(tmp_path / "wisdom"))
    yield
    m.kl_set_wisdom_dir(None)


def make_grids(shapes, dtypes, bcs, seed=0):
    m = kl()
    out = []
    for n, (shape, dt, bc) in enumerate(zip(shapes, dtypes, bcs)):
        g = m.Grid(*shape, dtype=dt, bc=bc)
        f = [g.full() for _ in range(3)]
        m.kl_generate_fields(g, seed + n, *f)
        m.kl_fill_ghosts(g, *f)
        t = [g.zeros_interior(fill=-3.0) for _ in range(3)]
        out.append((g, f, t))
    return out


def plain(m, grids, visc):
    res = []
    for g, f, _ in grids:
        t = [g.zeros_interior(fill=-3.0) for _ in range(3)]
        m.kl_advec_u(g, t[0], *f)
        m.kl_diff_uvw(g, *t, *f, visc)
        res.append([x.cpu().numpy() for x in t])
    return res


SHAPES = [(64, 64, 64), (32, 96, 40), (192, 32, 17), (128, 128, 8), (96, 20, 33), (256, 8, 12),
          (40, 24, 6), (33, 7, 5)]


def test_batch_bitwise_equals_single_grid_launches():
    m = kl()
    dts = [0, 1, 0, 1, 0, 0, 1, 0]
    bcs = [0, 2, 0, 0, 1, 2, 0, 2]
    grids = make_grids(SHAPES, dts, bcs, seed=11)
    visc = 1e-5
    ref = plain(m, grids, visc)
    b = m.kl_batch_create([g for g, _, _ in grids], [f + t for _, f, t in grids], visc, True)
    try:
        nk, nt = m.kl_batch_info(b)
        assert nk >= 2 and nt >= len(grids)
        for rep in range(3):
            for g, _, t in grids:  # garbage in the interiors: the graph zeroes them
                for x in t:
                    g.interior(x).fill_(9.0)
            m.kl_batch_run(b)
            torch.cuda.synchronize()
            # eager work between replays
            torch.cuda.synchronize()
            for (g, _, t), r in zip(grids, ref):
                mask = outside_interior_mask(g)
                for x, y in zip(t, r):
                    got = x.cpu().numpy()
                    assert np.array_equal(got, y), f"replay {rep}: batched result differs for {g.itot}x{g.jtot}x{g.ktot}"
                    assert np.all(got[mask] == -3.0)
    finally:
        m.kl_batch_destroy(b)


def test_batch_matches_oracle():
    m = kl()
    cases = [Case(48, 40, 24, 0, seed=5), Case(64, 16, 20, 1, bc=2, seed=6)]
    grids = []
    for c in cases:
        t = [c.g.zeros_interior(fill=0.0) for _ in range(3)]
        grids.append((c, t))
    b = m.kl_batch_create([c.g for c, _ in grids], [c.dev + t for c, t in grids], cases[0].visc, True)
    m.kl_batch_run(b)
    torch.cuda.synchronize()
    m.kl_batch_destroy(b)
    for c, t in grids:
        adv, du, dv, dw = c.oracle_tendencies()
        dtype = c.g.dtype
        eps = float(np.finfo(np.float32 if dtype == 0 else np.float64).eps)
        for n, (x, r) in enumerate(zip(t, (adv + du, dv, dw))):
            err = np.max(np.abs(c.gpu_interior(x) - r))
            if n == 0:
                # ut = advec_u + diff_u: each kernel's output within TOL of its
                # own maximum, then one rounding of the sum
                bound = TOL[dtype] * (np.max(np.abs(adv)) + np.max(np.abs(du))) + eps * np.max(np.abs(r))
            else:
                bound = TOL[dtype] * np.max(np.abs(r))
            assert err <= bound, f"output {n}: error {err:.3e} > {bound:.3e}"


def test_batched_workload_shapes_and_equality():
    """The 48 + 8 grid workload (FP32) in one graph equals per-grid launches."""
    m = kl()
    shapes = inputs.batch_shapes(3)
    assert len(shapes) == 56 and shapes[-1] == (256, 256, 32)
    assert all(s in inputs.BATCH_SIZES for sh in shapes[:48] for s in sh)
    grids = make_grids(shapes, [0] * 56, [0] * 56, seed=300)
    ref = plain(m, grids, 1e-5)
    b = m.kl_batch_create([g for g, _, _ in grids], [f + t for _, f, t in grids], 1e-5, True)
    m.kl_batch_run(b)
    torch.cuda.synchronize()
    nk, nt = m.kl_batch_info(b)
    m.kl_batch_destroy(b)
    assert nk <= 16
    for (g, _, t), r in zip(grids, ref):
        for x, y in zip(t, r):
            assert np.array_equal(x.cpu().numpy(), y)


def test_batch_rejects_bad_arguments():
    m = kl()
    g = m.Grid(16, 16, 16)
    f = [g.full() for _ in range(6)]
    with pytest.raises(m.KLError):
        m.kl_batch_create([g], [f[:5] + [None]], 1e-5, True)


def test_batch_tune_records_and_reuses_the_winner(tmp_path):
    """kl_batch_tune times the per-grid selection and every persistent
    configuration on the batch itself, appends the winner per dtype under the
    batch's signature, and a new batch of the same grids (in another order)
    takes it; the results stay bitwise those of single-grid launches."""
    import json
    m = kl()
    shapes = [(64, 32, 40), (32, 64, 24), (128, 16, 16), (96, 40, 20), (48, 24, 12), (40, 40, 8)]
    dts = [0, 0, 0, 0, 1, 1]
    bcs = [0, 2, 1, 0, 0, 2]
    grids = make_grids(shapes, dts, bcs, seed=41)
    wd = tmp_path / "wtune"
    b = m.kl_batch_create([g for g, _, _ in grids], [f + t for _, f, t in grids], 1e-5, True)
    try:
        res = m.kl_batch_tune(b, wd, 30.0)
    finally:
        m.kl_batch_destroy(b)
    assert res[0][0] == -1 and res[0][1] > 0, "the per-grid selection is timed first"
    assert all(ms > 0 for _, ms in res), "a configuration gave different bits"
    recs = [json.loads(x) for x in (wd / "advec_diff_batch.wisdom").read_text().splitlines()]
    assert sorted(r["dtype"] for r in recs) == ["f32", "f64"]
    assert {r["grids"] for r in recs} == {4, 2}
    m.kl_set_wisdom_dir(str(wd))
    order = [3, 0, 5, 2, 4, 1]
    regrids = [grids[n] for n in order]
    ref = plain(m, regrids, 1e-5)
    b = m.kl_batch_create([g for g, _, _ in regrids], [f + t for _, f, t in regrids], 1e-5, True)
    try:
        groups = m.kl_batch_groups(b)
        for r in recs:
            if r["variant"] != "per_grid":
                dt = 0 if r["dtype"] == "f32" else 1
                assert any(d == dt and name == r["variant"] for d, name, _ in groups), (r, groups)
        m.kl_batch_run(b)
        torch.cuda.synchronize()
        for (g, _, t), rr in zip(regrids, ref):
            for x, y in zip(t, rr):
                assert np.array_equal(x.cpu().numpy(), y)
    finally:
        m.kl_batch_destroy(b)


def test_batch_graph_with_ghost_fill_zeroing_and_sums():
    """kl_batch_create_ex with every step: [ghost fill] -> [tendencies := 0]
    -> the fused groups -> [conservation sums].  On every replay (with eager
    work between replays that undoes what the graph did) u, v, w come out
    bitwise as kl_fill_ghosts leaves them, the tendencies bitwise those of the
    single-grid launches on the filled fields, and each grid's sums bitwise
    those of kl_reduce_fp64(what = 0) on them."""
    m = kl()
    dts = [0, 1, 0, 1, 0, 0, 1, 0]
    bcs = [0, 2, 0, 0, 1, 2, 0, 1]
    visc = 1e-5
    grids, ref_f, ref_t, ref_s = [], [], [], []
    for n, (shape, dt, bc) in enumerate(zip(SHAPES, dts, bcs)):
        g = m.Grid(*shape, dtype=dt, bc=bc)
        f = [g.full() for _ in range(3)]  # ghosts left NaN: only the graph's fill sets them
        m.kl_generate_fields(g, 40 + n, *f)
        t = [g.zeros_interior(fill=-3.0) for _ in range(3)]
        rf = [x.clone() for x in f]
        m.kl_fill_ghosts(g, *rf)
        rt = [g.zeros_interior(fill=-3.0) for _ in range(3)]
        m.kl_advec_u(g, rt[0], *rf)
        m.kl_diff_uvw(g, *rt, *rf, visc)
        rs = torch.zeros(3, dtype=torch.float64, device="cuda")
        m.kl_reduce_fp64(g, 0, *rt, rs)
        grids.append((g, f, t))
        ref_f.append([x.cpu().numpy() for x in rf])
        ref_t.append([x.cpu().numpy() for x in rt])
        ref_s.append(rs.cpu().numpy())
    sums = torch.full((3 * len(grids),), np.nan, dtype=torch.float64, device="cuda")
    with pytest.raises(m.KLError):
        m.kl_batch_create_ex([g for g, _, _ in grids], [f + t for _, f, t in grids], visc, 8)
    with pytest.raises(m.KLError):
        m.kl_batch_create_ex([g for g, _, _ in grids], [f + t for _, f, t in grids], visc, m.BATCH_SUMS)
    flags = m.BATCH_FILL_GHOSTS | m.BATCH_ZERO_TENDENCIES | m.BATCH_SUMS
    b = m.kl_batch_create_ex([g for g, _, _ in grids], [f + t for _, f, t in grids], visc, flags, sums)
    try:
        nk, _ = m.kl_batch_info(b)
        assert nk >= 4  # fill, zero, at least one fused group, sums
        for rep in range(3):
            # undo the previous replay: ghosts back to NaN, tendencies to junk
            for g, f, t in grids:
                for x in f:
                    keep = g.interior(x).clone()
                    g.box(x).fill_(np.nan)
                    g.interior(x).copy_(keep)
                for x in t:
                    g.interior(x).fill_(7.0)
            sums.fill_(np.nan)
            torch.cuda.synchronize()
            m.kl_batch_run(b)
            torch.cuda.synchronize()
            s = sums.cpu().numpy()
            for n, (g, f, t) in enumerate(grids):
                for q in range(3):
                    assert np.array_equal(f[q].cpu().numpy(), ref_f[n][q], equal_nan=True), (rep, n, "field", q)
                    assert np.array_equal(t[q].cpu().numpy(), ref_t[n][q], equal_nan=True), (rep, n, "tendency", q)
                assert np.array_equal(s[3 * n:3 * n + 3], ref_s[n]), (rep, n, s[3 * n:3 * n + 3], ref_s[n])
    finally:
        m.kl_batch_destroy(b)
