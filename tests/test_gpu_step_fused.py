"""Fused time step: bitwise the same state (ghost cells included) as the
separate kernels of kl_step, for every fused configuration; inputs untouched;
row and tail padding of the outputs never written."""
import numpy as np
import pytest
import torch

from gpu_util import TOL, Case, rel_err

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


# 260, 130 and 65 leave one active lane in the last x tile at 4, 2 and 1 points per lane
SHAPES = [(64, 48, 20), (37, 23, 19), (256, 12, 9), (5, 4, 6), (128, 64, 33), (96, 3, 2), (260, 6, 9), (130, 5, 11),
          (65, 4, 7)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_fused_step_bitwise_equals_kl_step(dtype, bc, shape):
    m = kl()
    g = m.Grid(*shape, dtype=dtype, bc=bc)
    f = [g.full() for _ in range(3)]
    m.kl_generate_fields(g, 21, *f)
    m.kl_fill_ghosts(g, *f)
    visc, dt = 1e-3, 2e-3
    ref = [x.clone() for x in f]
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    m.kl_step(g, visc, dt, *ref, *tend)
    refb = [g.box(x).cpu().numpy() for x in ref]
    before = [x.clone() for x in f]
    n = m.kl_num_variants(m.STEP, dtype)
    ran = 0
    for idx in range(n):
        out = [g.full() for _ in range(3)]
        fields = f + out
        if not m.kl_variant_eligible(g, m.STEP, idx, fields):
            continue
        m.kl_launch_variant_dt(g, m.STEP, idx, fields, visc, dt)
        name = m.kl_variant_name(m.STEP, dtype, idx)
        for a, b in zip(out, refb):
            assert np.array_equal(g.box(a).cpu().numpy(), b), name
            assert padding_untouched(g, a), f"{name} wrote a padding cell"
        ran += 1
    assert ran >= 1
    for a, b in zip(f, before):
        assert torch.equal(torch.nan_to_num(a, 123.0), torch.nan_to_num(b, 123.0)), "fused step modified its input"
    # the selected path through kl_step_fused
    out = [g.full() for _ in range(3)]
    m.kl_step_fused(g, visc, dt, *f, *out)
    for a, b in zip(out, refb):
        assert np.array_equal(g.box(a).cpu().numpy(), b)
        assert padding_untouched(g, a)


def padding_untouched(g, t):
    """Every cell outside the ghost box of a NaN-filled output is still NaN
    (the box of a copy is set to NaN, then every cell must be NaN)."""
    x = t.clone()
    g.box(x).fill_(float("nan"))
    return bool(torch.isnan(x).all())


def test_fused_steps_ping_pong_match_oracle():
    import oracle
    m = kl()
    c = Case(48, 32, 24, 1, bc=0, seed=17)
    g = c.g
    visc, dt = 1e-3, 1e-3
    a = c.dev
    b = [g.full() for _ in range(3)]
    for _ in range(4):
        m.kl_step_fused(g, visc, dt, *a, *b)
        a, b = b, a
    host = [h.copy() for h in c.host]
    tmp = [np.zeros(g.alloc) for _ in range(3)]
    for _ in range(4):
        oracle.step(c.og, visc, dt, *host, *tmp)
    # 4 FP64 steps: each adds at most dt*TOL*max|ft| of tendency error and one
    # rounding of the state, far inside the kernel tolerance
    for d, h in zip(a, host):
        assert rel_err(c.gpu_interior(d), c.interior_np(h)) <= TOL[1]


def test_fused_step_rejects_aliasing():
    m = kl()
    g = m.Grid(16, 16, 8)
    f = [g.full() for _ in range(3)]
    with pytest.raises(m.KLError):
        m.kl_step_fused(g, 1e-5, 1e-3, *f, f[0], f[1], f[2])
