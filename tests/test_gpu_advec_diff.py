"""kl_advec_diff, the fused advec_u + diff_uvw pass, through the C ABI.

It must match the oracle's advec_u followed by its diff_uvw (accumulated in
that order into the same tendencies) to the kernel tolerance, never write
outside the interior, and equal kl_advec_u followed by kl_diff_uvw bit for
bit in every compiled configuration (the additions are made and rounded in
the same order)."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2303_12374_amd import inputs
from gpu_util import TOL, Case, accumulate_bound, outside_interior_mask, rel_err

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHAPES = [(64, 64, 64), (37, 23, 19), (5, 4, 6), (1, 1, 2), (130, 7, 33)]


def kl():
    from paper_2303_12374_amd import kl as m
    return m


@pytest.fixture(autouse=True)
def no_wisdom(tmp_path):
    m = kl()
    m.kl_set_wisdom_dir(str(tmp_path / "wisdom"))
    yield
    m.kl_set_wisdom_dir(None)


def oracle_pair(c, init=None):
    """Oracle: tendencies (init, else 0) += advec_u, then += diff_uvw."""
    og = c.og
    bufs = []
    for n in range(3):
        b = np.zeros(og.alloc)
        if init is not None:
            inputs.padded_view(b, og.itot, og.jtot, og.ktot, og.off, og.js, og.ks)[
                1:og.ktot + 1, 1:og.jtot + 1, 1:og.itot + 1] = init[n]
        bufs.append(b)
    oracle.advec_u(og, bufs[0], *c.host)
    oracle.diff_uvw(og, bufs[0], bufs[1], bufs[2], *c.host, c.visc_eff)
    return [c.interior_np(b) for b in bufs]


@pytest.mark.parametrize("layout", ["kl", "plain"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_advec_diff_matches_oracle(dtype, bc, shape, layout):
    m = kl()
    lay = None if layout == "kl" else inputs.plain_layout(*shape)
    c = Case(*shape, dtype, bc=bc, seed=sum(shape) + 5, layout=lay)
    g = c.g
    sentinel = 7.0
    ts = [g.zeros_interior(fill=sentinel) for _ in range(3)]
    m.kl_advec_diff(g, *ts, *c.dev, c.visc)
    ref = oracle_pair(c)
    mask = outside_interior_mask(g)
    for name, t, r in zip(("ut", "vt", "wt"), ts, ref):
        got = c.gpu_interior(t)
        assert np.all(np.isfinite(got)), f"{name}: non-finite output"
        err = rel_err(got, r)
        assert err <= TOL[dtype], f"{name}: rel err {err:.3e} > {TOL[dtype]}"
        assert np.all(t.cpu().numpy()[mask] == sentinel), f"{name}: wrote outside the interior"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_advec_diff_accumulates(dtype):
    """The pass adds to tendencies already present: against the oracle's sums
    of the initial values and its tendencies, with the bound of two
    accumulating kernels (the tolerance of each, and one rounding each)."""
    m = kl()
    c = Case(40, 24, 12, dtype, seed=8)
    g = c.g
    rng = np.random.default_rng(2)
    npd = m.NP_DTYPE[dtype]
    init = [rng.uniform(-3, 3, (g.ktot, g.jtot, g.itot)).astype(npd).astype(np.float64) for _ in range(3)]
    ts = [g.upload(x, fill=0.0) for x in init]
    m.kl_advec_diff(g, *ts, *c.dev, c.visc)
    zero = oracle_pair(c)
    ref = oracle_pair(c, init)
    for n, (t, r, z) in enumerate(zip(ts, ref, zero)):
        err = np.max(np.abs(c.gpu_interior(t) - r))
        bound = 2 * accumulate_bound(z, r, dtype)
        assert err <= bound, f"output {n}: accumulate error {err:.3e} > {bound:.3e}"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 40, 37), (256, 3, 70), (260, 6, 9), (130, 5, 11), (65, 4, 7)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bc", [0, 2], ids=["zerograd", "zperiodic"])
def test_every_configuration_equals_separate_kernels(bc, shape, dtype):
    """Every configuration of the fused pass, on non-zero initial tendencies,
    equals the default advec_u followed by the default diff_uvw bit for bit,
    cells outside the interior included (they keep their sentinel)."""
    m = kl()
    c = Case(*shape, dtype, bc=bc, seed=13)
    g = c.g
    rng = np.random.default_rng(4)
    init = [rng.uniform(-2, 2, (g.ktot, g.jtot, g.itot)) for _ in range(3)]
    ref = [g.upload(x, fill=-5.0) for x in init]
    m.kl_launch_variant(g, m.ADVEC_U, 0, c.dev + ref, c.visc)
    m.kl_launch_variant(g, m.DIFF_UVW, 0, c.dev + ref, c.visc)
    ref = [r.cpu().numpy() for r in ref]
    ran = 0
    for idx in range(m.kl_num_variants(m.ADVEC_DIFF, dtype)):
        outs = [g.upload(x, fill=-5.0) for x in init]
        fields = c.dev + outs
        if not m.kl_variant_eligible(g, m.ADVEC_DIFF, idx, fields):
            continue
        m.kl_launch_variant(g, m.ADVEC_DIFF, idx, fields, c.visc)
        for q, (o, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(o.cpu().numpy(), r), \
                f"{m.kl_variant_name(m.ADVEC_DIFF, dtype, idx)} output {q} differs from the separate kernels"
        ran += 1
    assert ran >= (8 if shape[0] % 4 == 0 else 2)


def test_tuning_the_fused_pass_writes_a_selectable_record(tmp_path):
    """kl_tune on the fused pass: every configuration passes the bitwise check
    against the default, and the record it appends is the one selected."""
    m = kl()
    c = Case(128, 64, 32, 0, seed=3)
    g = c.g
    outs = [g.zeros_interior(fill=0.0) for _ in range(3)]
    wd = tmp_path / "wisdom"
    res = m.kl_tune(g, c.dev + outs, m.TUNE_ADVEC_DIFF, wd, 20.0)
    assert res and all(ms > 0 for _, ms in res), "a configuration failed the bitwise check"
    best = min(res, key=lambda x: x[1])[0]
    m.kl_set_wisdom_dir(str(wd))
    assert m.kl_selected_variant(g, m.ADVEC_DIFF) == best
    assert (wd / "advec_diff.wisdom").exists()


@pytest.mark.parametrize("shape", [(512, 512, 512), (1024, 1024, 128)], ids=["512cube", "1024x1024x128"])
def test_full_size_selected_equals_separate(shape):
    """At the benchmark's sizes (FP32), the configuration the committed wisdom
    selects equals the separate advec_u and diff_uvw (default configurations)
    bitwise on the whole interior, and writes nothing outside it."""
    m = kl()
    m.kl_set_wisdom_dir(os.path.join(ROOT, "wisdom"))
    try:
        g = m.Grid(*shape, dtype=0, bc=0)
        dev = [g.full(0.0) for _ in range(3)]
        m.kl_generate_fields(g, 21, *dev)
        m.kl_fill_ghosts(g, *dev)
        a = [g.zeros_interior(fill=-5.0) for _ in range(3)]
        m.kl_advec_diff(g, *a, *dev, 1e-5)
        b = [g.zeros_interior(fill=0.0) for _ in range(3)]
        m.kl_launch_variant(g, m.ADVEC_U, 0, dev + b, 1e-5)
        m.kl_launch_variant(g, m.DIFF_UVW, 0, dev + b, 1e-5)
        h = torch.zeros(6, dtype=torch.int64, device="cuda")
        for q in range(3):
            m.kl_hash_interior(g, a[q], h[2 * q:2 * q + 1])
            m.kl_hash_interior(g, b[q], h[2 * q + 1:2 * q + 2])
        hh = h.cpu().numpy()
        for q in range(3):
            assert hh[2 * q] == hh[2 * q + 1], f"output {q}: selected fused configuration differs"
            x = a[q].clone()
            g.interior(x).fill_(-5.0)
            assert bool((x == -5.0).all()), f"output {q} written outside the interior"
            del x
    finally:
        m.kl_set_wisdom_dir(None)
