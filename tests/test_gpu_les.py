"""GPU parity of the paper's own schemes: advec_u_2i5 (fifth-order
interpolated advection of u, three ghost cells in x and y) and diff_smag
(stress divergence with a cell-center eddy viscosity), through the C ABI,
against the CPU oracle on the same seeded inputs.  Bar: normwise relative
error <= 1e-12 (FP64) and <= 1e-5 (FP32) per output field; ghost fill
bitwise; every configuration bitwise equal to the default one."""
import numpy as np
import pytest
import torch

import oracle
from paper_2303_12374_amd import inputs
from gpu_util import TOL, accumulate_bound, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64, 64), (37, 23, 19), (5, 4, 6), (2, 3, 4), (1, 1, 2), (130, 7, 33)]
EVISC_MEAN = 2e-3
SENTINEL = -5.0


def kl():
    from paper_2303_12374_amd import kl as m
    return m


@pytest.fixture(autouse=True)
def no_wisdom(tmp_path):
    m = kl()
    m.kl_set_wisdom_dir(str(tmp_path / "wisdom"))
    yield
    m.kl_set_wisdom_dir(None)


class LesCase:
    """Device and oracle state of one grid with gc ghost cells in x and y."""

    def __init__(self, itot, jtot, ktot, dtype, bc=0, seed=0, gc=3, layout=None):
        m = kl()
        self.m = m
        self.g = m.Grid(itot, jtot, ktot, dtype=dtype, bc=bc, gc=gc, layout=layout)
        g = self.g
        npd = m.NP_DTYPE[dtype]
        fs = inputs.random_fields(seed, itot, jtot, ktot)
        fs.append(inputs.evisc_field(seed, itot, jtot, ktot, mean=EVISC_MEAN))
        self.fs = [np.ascontiguousarray(f.astype(npd)) for f in fs]   # what the GPU sees
        self.dev = [g.upload(f) for f in self.fs]
        m.kl_fill_ghosts(g, *self.dev[:3])
        m.kl_fill_scalar(g, self.dev[3])
        self.og = oracle.Grid(itot, jtot, ktot, g.off, g.js, g.ks, g.alloc, g.dxi, g.dyi,
                              g.dzi_h.astype(np.float64), g.dzhi_h.astype(np.float64), bc, gc)
        self.host = [inputs.embed(f.astype(np.float64), g.off, g.js, g.ks, g.alloc, gh=gc) for f in self.fs]
        oracle.fill_ghosts(self.og, *self.host[:3])
        oracle.fill_scalar(self.og, self.host[3])

    def zero_buf(self):
        og = self.og
        b = np.full(og.alloc, np.nan)
        self.interior_np(b)[...] = 0.0
        return b

    def interior_np(self, buf):
        og = self.og
        return inputs.interior_view(buf, og.itot, og.jtot, og.ktot, og.off, og.js, og.ks, og.gc)

    def oracle_advec(self):
        b = self.zero_buf()
        oracle.advec_u_2i5(self.og, b, *self.host[:3])
        return self.interior_np(b)

    def oracle_smag(self):
        bs = [self.zero_buf() for _ in range(3)]
        oracle.diff_smag(self.og, *bs, *self.host)
        return [self.interior_np(b) for b in bs]

    def gpu_interior(self, t):
        return self.g.interior(t).cpu().numpy().astype(np.float64)

    def outside_mask(self):
        g = self.g
        m = np.ones(g.alloc, bool)
        k = np.arange(1, g.ktot + 1)[:, None, None]
        j = np.arange(1, g.jtot + 1)[None, :, None]
        i = np.arange(1, g.itot + 1)[None, None, :]
        m[(g.off + i + j * g.js + k * g.ks).ravel()] = False
        return m


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
@pytest.mark.parametrize("shape", [(11, 6, 5), (2, 1, 3)], ids=lambda s: "x".join(map(str, s)))
def test_fill_three_ghost_cells_bitwise(dtype, bc, shape):
    c = LesCase(*shape, dtype, bc=bc, seed=4)
    for d, h in zip(c.dev, c.host):
        got = d.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, h, equal_nan=True), "ghost fill differs from the oracle"


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_les_tendencies_match_oracle(dtype, bc, shape):
    m = kl()
    c = LesCase(*shape, dtype, bc=bc, seed=sum(shape) + bc)
    g = c.g
    sentinel = 7.0
    adv = g.zeros_interior(fill=sentinel)
    ts = [g.zeros_interior(fill=sentinel) for _ in range(3)]
    m.kl_advec_u_2i5(g, adv, *c.dev[:3])
    m.kl_diff_smag(g, *ts, *c.dev)
    ref = [c.oracle_advec()] + c.oracle_smag()
    mask = c.outside_mask()
    for name, t, r in zip(("advec_u_2i5", "smag_u", "smag_v", "smag_w"), [adv] + ts, ref):
        got = c.gpu_interior(t)
        assert np.all(np.isfinite(got)), f"{name}: non-finite output (read of an unset cell?)"
        err = rel_err(got, r)
        assert err <= TOL[dtype], f"{name}: rel err {err:.3e} > {TOL[dtype]}"
        assert np.all(t.cpu().numpy()[mask] == sentinel), f"{name}: wrote outside the interior"


@pytest.mark.parametrize("shape", [(37, 23, 19), (64, 16, 8)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_les_unpadded_layout(dtype, shape):
    """The schemes on an unpadded layout (rows of itot+6 cells, no line
    alignment): every configuration that is eligible there (the default one
    at least) matches the oracle."""
    m = kl()
    lay = inputs.plain_layout(*shape, gh=3)
    c = LesCase(*shape, dtype, bc=0, seed=41, layout=lay)
    g = c.g
    ref = [c.oracle_advec()] + c.oracle_smag()
    mask = c.outside_mask()
    for kernel, nout in ((m.ADVEC_U_2I5, 1), (m.DIFF_SMAG, 3)):
        for idx in range(m.kl_num_variants(kernel, dtype)):
            outs = [g.zeros_interior(fill=SENTINEL) for _ in range(3)]
            fields = c.dev[:3] + outs + ([c.dev[3]] if kernel == m.DIFF_SMAG else [])
            if not m.kl_variant_eligible(g, kernel, idx, fields):
                continue
            m.kl_launch_variant(g, kernel, idx, fields)
            name = m.kl_variant_name(kernel, dtype, idx)
            r = ref[:1] if nout == 1 else ref[1:]
            for q in range(3):
                flat = outs[q].cpu().numpy()
                assert np.all(flat[mask] == SENTINEL), f"{name} output {q}: wrote outside the interior"
                if q < nout:
                    err = rel_err(c.gpu_interior(outs[q]), r[q])
                    assert err <= TOL[dtype], f"{name} output {q}: {err:.3e}"
                else:
                    assert np.all(flat[~mask] == 0.0), f"{name}: wrote output slot {q} it does not own"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_les_tendencies_accumulate(dtype):
    m = kl()
    c = LesCase(40, 24, 12, dtype, seed=8)
    g = c.g
    rng = np.random.default_rng(1)
    init = [rng.uniform(-3, 3, (g.ktot, g.jtot, g.itot)) for _ in range(4)]
    ts = [g.upload(x, fill=0.0) for x in init]
    m.kl_advec_u_2i5(g, ts[0], *c.dev[:3])
    m.kl_diff_smag(g, ts[1], ts[2], ts[3], *c.dev)
    ref = [c.oracle_advec()] + c.oracle_smag()
    npd = m.NP_DTYPE[dtype]
    for n, (t, r, x0) in enumerate(zip(ts, ref, init)):
        expect = x0.astype(npd).astype(np.float64) + r
        err = np.max(np.abs(c.gpu_interior(t) - expect))
        bound = accumulate_bound(r, expect, dtype)
        assert err <= bound, f"output {n}: accumulate error {err:.3e} > {bound:.3e}"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_diff_smag_on_one_ghost_cell_grid(dtype):
    """diff_smag needs one ghost cell: it runs on the library's gc = 1 layout."""
    m = kl()
    c = LesCase(48, 20, 10, dtype, bc=0, seed=12, gc=1)
    g = c.g
    ts = [g.zeros_interior(fill=0.0) for _ in range(3)]
    m.kl_diff_smag(g, *ts, *c.dev)
    for n, (t, r) in enumerate(zip(ts, c.oracle_smag())):
        err = rel_err(c.gpu_interior(t), r)
        assert err <= TOL[dtype], f"smag {n} on gc=1: rel err {err:.3e}"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_pair_tuning_of_diff_smag_on_one_ghost_cell_grid(dtype, tmp_path):
    """In pair mode diff_smag is timed after advec_u_2i5, which needs three
    ghost cells; on a one-ghost-cell grid it is tuned on its own instead of
    failing."""
    m = kl()
    c = LesCase(48, 20, 10, dtype, bc=0, seed=12, gc=1)
    g = c.g
    ts = [g.zeros_interior(fill=0.0) for _ in range(3)]
    wdir = tmp_path / "pairw"
    timings = m.kl_tune(g, c.dev[:3] + ts + [c.dev[3]], m.TUNE_DIFF_SMAG | m.TUNE_PAIR, wdir, budget_s=5.0)
    assert timings and timings[0][0] == 0 and timings[0][1] > 0
    lines = (wdir / "diff_smag.wisdom").read_text().splitlines()
    assert len(lines) == 1 and '"after_advec":1' in lines[0]


@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 40, 37), (256, 3, 70), (260, 6, 9), (130, 5, 11), (65, 4, 7)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("kernel", [3, 4], ids=["advec_u_2i5", "diff_smag"])
def test_every_les_configuration_bitwise_equal(kernel, dtype, shape):
    """Every eligible configuration writes exactly the default
    configuration's bits into the interior of its outputs and leaves every
    other cell (ghosts, row padding, the untouched output slots) holding its
    sentinel.  260, 130 and 65 leave one active lane in the last x tile."""
    m = kl()
    c = LesCase(*shape, dtype, seed=3)
    g = c.g
    mask = c.outside_mask()
    n = m.kl_num_variants(kernel, dtype)
    nout = 1 if kernel == m.ADVEC_U_2I5 else 3
    ref = None
    ran = 0
    for idx in range(n):
        outs = [g.zeros_interior(fill=SENTINEL) for _ in range(3)]
        fields = c.dev[:3] + outs + ([c.dev[3]] if kernel == m.DIFF_SMAG else [])
        if not m.kl_variant_eligible(g, kernel, idx, fields):
            continue
        m.kl_launch_variant(g, kernel, idx, fields)
        name = m.kl_variant_name(kernel, dtype, idx)
        got = [o.cpu().numpy() for o in outs]
        for q, a in enumerate(got):
            assert np.all(a[mask] == SENTINEL), f"configuration {name} output {q}: wrote outside the interior"
        for a in got[nout:]:
            assert np.all(a[~mask] == 0.0), f"configuration {name}: wrote an output slot it does not own"
        if ref is None:
            assert idx == 0
            ref = got
            # the default configuration itself agrees with the oracle
            r = [c.oracle_advec()] if nout == 1 else c.oracle_smag()
            for q in range(nout):
                assert rel_err(c.gpu_interior(outs[q]), r[q]) <= TOL[dtype]
        else:
            for q in range(nout):
                assert np.array_equal(got[q], ref[q]), f"configuration {name} output {q} differs"
        ran += 1
    assert ran >= 1
