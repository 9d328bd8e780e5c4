"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle on
the same seeded inputs.  Bar: normwise relative error <= 1e-12 (FP64) and
<= 1e-5 (FP32) per output field, bitwise equality of ghost fill, of the
reductions' inputs and of every configuration against the default one."""
import numpy as np
import pytest

import oracle
from paper_2303_12374_amd import inputs
from gpu_util import TOL, Case, accumulate_bound, outside_interior_mask, rel_err

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
def test_fill_ghosts_bitwise(dtype, bc):
    c = Case(11, 6, 5, dtype, bc=bc, seed=4)
    for d, h in zip(c.dev, c.host):
        got = d.cpu().numpy().astype(np.float64)
        assert np.array_equal(got, h, equal_nan=True), "ghost fill differs from the oracle"


@pytest.mark.parametrize("layout", ["kl", "plain"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("bc", [0, 2], ids=["zerograd", "zperiodic"])
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_tendencies_match_oracle(dtype, bc, shape, layout):
    m = kl()
    lay = None if layout == "kl" else inputs.plain_layout(*shape)
    c = Case(*shape, dtype, bc=bc, seed=sum(shape), layout=lay)
    g = c.g
    sentinel = 7.0
    adv = g.zeros_interior(fill=sentinel)
    ut, vt, wt = (g.zeros_interior(fill=sentinel) for _ in range(3))
    m.kl_advec_u(g, adv, *c.dev)
    m.kl_diff_uvw(g, ut, vt, wt, *c.dev, c.visc)
    ref = c.oracle_tendencies()
    mask = outside_interior_mask(g)
    for name, t, r in zip(("advec_u", "diff_u", "diff_v", "diff_w"), (adv, ut, vt, wt), ref):
        got = c.gpu_interior(t)
        assert np.all(np.isfinite(got)), f"{name}: non-finite output (read of an unset cell?)"
        err = rel_err(got, r)
        assert err <= TOL[dtype], f"{name}: rel err {err:.3e} > {TOL[dtype]}"
        flat = t.cpu().numpy()
        assert np.all(flat[mask] == sentinel), f"{name}: wrote outside the interior"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_tendencies_accumulate(dtype):
    """Kernels add to the tendency already present."""
    m = kl()
    c = Case(40, 24, 12, dtype, seed=8)
    g = c.g
    rng = np.random.default_rng(1)
    init = [rng.uniform(-3, 3, (g.ktot, g.jtot, g.itot)) for _ in range(4)]
    ts = [g.upload(x, fill=0.0) for x in init]
    m.kl_advec_u(g, ts[0], *c.dev)
    m.kl_diff_uvw(g, ts[1], ts[2], ts[3], *c.dev, c.visc)
    ref = c.oracle_tendencies()
    npd = m.NP_DTYPE[dtype]
    for n, (t, r, x0) in enumerate(zip(ts, ref, init)):
        expect = x0.astype(npd).astype(np.float64) + r
        if n == 3 and c.g.bc != 2:
            expect[0] = x0[0].astype(npd)
        err = np.max(np.abs(c.gpu_interior(t) - expect))
        bound = accumulate_bound(r, expect, dtype)
        assert err <= bound, f"output {n}: accumulate error {err:.3e} > {bound:.3e}"


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("kernel", [0, 1], ids=["advec_u", "diff_uvw"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 40, 37), (256, 3, 70), (260, 6, 9), (130, 5, 11), (65, 4, 7)],
                         ids=lambda s: "x".join(map(str, s)))
def test_every_configuration_bitwise_equal(kernel, dtype, shape):
    """All compiled configurations give bit-identical tendencies (same
    per-point arithmetic), and never write outside the interior.  260, 130
    and 65 leave one active lane in the last x tile at 4, 2 and 1 points per
    lane (its right edge value then comes from lane 1)."""
    m = kl()
    c = Case(*shape, dtype, seed=3)
    g = c.g
    mask = outside_interior_mask(g)
    ref = None
    n = m.kl_num_variants(kernel, dtype)
    ran = 0
    for idx in range(n):
        outs = [g.zeros_interior(fill=-5.0) for _ in range(3)]
        fields = c.dev + outs
        if not m.kl_variant_eligible(g, kernel, idx, fields):
            continue
        m.kl_launch_variant(g, kernel, idx, fields, c.visc)
        got = [o.cpu().numpy() for o in outs]
        if ref is None:
            ref = got
            assert idx == 0
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"configuration {m.kl_variant_name(kernel, dtype, idx)} differs"
            assert np.all(a[mask] == -5.0)
        ran += 1
    assert ran > 4 if shape[0] % 4 == 0 else ran >= 1


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
def test_step_matches_oracle(dtype, bc):
    m = kl()
    c = Case(48, 20, 16, dtype, bc=bc, seed=21)
    g = c.g
    dt = 1e-3
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    for _ in range(3):
        m.kl_step(g, c.visc, dt, *c.dev, *tend)
    host = [h.copy() for h in c.host]
    tmp = [np.zeros(g.alloc) for _ in range(3)]
    npd = m.NP_DTYPE[dtype]
    for _ in range(3):
        oracle.step(c.og, c.visc_eff, float(npd(dt)), *host, *tmp)
        if dtype == 0:  # the FP32 path rounds the state to FP32 after every step
            host = [h.astype(np.float32).astype(np.float64) for h in host]
    box = lambda b: inputs.padded_view(b, g.itot, g.jtot, g.ktot, g.off, g.js, g.ks)
    # The state is checked at the kernel tolerance, unwidened.  Each step adds
    # dt times the kernels' tendency error (a few ulps of max|ft|) and one
    # rounding of the state on each side, so the state error after 3 steps
    # is a few eps of max|f|.  A fault in the step itself (stale ghosts, a
    # wrong wall rule, a lost term) moves the state by O(dt*ft), far above
    # TOL.  The strict bound on one step's increment is checked by
    # test_step_increment_matches_oracle.
    for d, h in zip(c.dev, host):
        flat = d.cpu().numpy()
        got = box(flat.astype(np.float64))
        ref = box(h)
        assert rel_err(got, ref) <= TOL[dtype]
        outside_box = np.ones(g.alloc, bool)
        box(outside_box)[...] = False
        assert np.all(np.isnan(flat[outside_box])), "the step wrote a padding cell"
    chk = [d.clone() for d in c.dev]
    m.kl_fill_ghosts(g, *chk)
    for a, b in zip(chk, c.dev):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True), "Euler step left ghosts stale"


@pytest.mark.parametrize("bc", [0, 1, 2], ids=["zerograd", "nopen", "zperiodic"])
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_step_increment_matches_oracle(dtype, bc):
    """The change of the state over one step equals dt * oracle tendencies on
    every point the step advances; with z walls the wall faces of w follow
    the boundary rule instead (w_1 = w_2 and w_{ktot+1} = w_ktot, or 0)."""
    m = kl()
    c = Case(32, 16, 10, dtype, bc=bc, seed=5 + bc)
    g = c.g
    dt = 1e-3
    before = [c.gpu_interior(d) for d in c.dev]
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    m.kl_step(g, c.visc, dt, *c.dev, *tend)
    adv, du, dv, dw = c.oracle_tendencies()
    npd = m.NP_DTYPE[dtype]
    dte = float(npd(dt))
    eps = float(np.finfo(npd).eps)
    k0 = 0 if bc == 2 else 1  # first advanced w level, 0-based in the interior view
    for n, (d, b, r) in enumerate(zip(c.dev, before, (adv + du, dv, dw))):
        new = c.gpu_interior(d)
        inc = new - b
        if n == 2:
            inc, r, newc = inc[k0:], r[k0:], new[k0:]
        else:
            newc = new
        # tendency error at the kernel tolerance (the u tendency is the sum
        # of two kernels' outputs) plus the roundings of dt*ft and f + dt*ft
        rt = np.max(np.abs(dte * adv)) + np.max(np.abs(dte * du)) if n == 0 else np.max(np.abs(dte * r))
        bound = TOL[dtype] * rt + eps * (np.max(np.abs(newc)) + np.max(np.abs(dte * r)))
        err = np.max(np.abs(inc - dte * r))
        assert err <= bound, f"field {n}: increment error {err:.3e} > {bound:.3e}"
    if bc != 2:
        wb = g.box(c.dev[2]).cpu().numpy().astype(np.float64)
        if bc == 0:
            assert np.array_equal(wb[1], wb[2]) and np.array_equal(wb[g.ktot + 1], wb[g.ktot])
        else:
            assert np.all(wb[1] == 0.0) and np.all(wb[g.ktot + 1] == 0.0)


@pytest.mark.parametrize("shape", [(70, 33, 21), (64, 33, 21), (1024, 3, 4)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_reductions_match_oracle(dtype, shape):
    """itot = 70 takes the one-point-per-thread path; 64 and 1024 the 16-byte
    vector path (several rows per pass at 64; at 1024 a row is one pass or,
    in FP64, two chunks per thread)."""
    import torch
    m = kl()
    c = Case(*shape, dtype, bc=0, seed=12)
    g = c.g
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    m.kl_reduce_fp64(g, 1, *c.dev, out)
    got = out.cpu().numpy()
    for n, h in enumerate(c.host):
        ref = oracle.checksums(c.og, h)
        x = c.interior_np(h)
        assert abs(got[3 * n] - ref[0]) <= 1e-12 * np.sum(np.abs(x))
        assert abs(got[3 * n + 1] - ref[1]) <= 1e-12 * ref[1]
        assert got[3 * n + 2] == ref[2]
    # conservation sums of oracle-free inputs: tendencies = the fields themselves
    out3 = torch.zeros(3, dtype=torch.float64, device="cuda")
    m.kl_reduce_fp64(g, 0, *c.dev, out3)
    ref = oracle.conservation(c.og, *c.host)
    scale = sum(np.sum(np.abs(c.interior_np(h))) for h in c.host) * np.max(1.0 / c.og.dzi)
    assert np.max(np.abs(out3.cpu().numpy() - ref)) <= 1e-12 * scale
    # bitwise reproducible
    out_b = torch.zeros(9, dtype=torch.float64, device="cuda")
    m.kl_reduce_fp64(g, 1, *c.dev, out_b)
    assert torch.equal(out, out_b)


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
def test_device_generator_matches_numpy(dtype):
    """kl_generate_fields reproduces the host recipe bit for bit."""
    m = kl()
    g = m.Grid(45, 17, 9, dtype=dtype)
    dev = [g.full() for _ in range(3)]
    m.kl_generate_fields(g, 1234, *dev)
    ref = inputs.random_fields(1234, 45, 17, 9)
    for d, r in zip(dev, ref):
        assert np.array_equal(g.interior(d).cpu().numpy(), r.astype(m.NP_DTYPE[dtype]))


def test_hash_detects_single_bit_change():
    import torch
    m = kl()
    c = Case(33, 9, 7, 0, seed=2)
    g = c.g
    h = torch.zeros(2, dtype=torch.int64, device="cuda")
    m.kl_hash_interior(g, c.dev[0], h[0:1])
    x = c.dev[0].clone()
    xi = g.interior(x)
    xi[3, 4, 5] = torch.nextafter(xi[3, 4, 5], torch.tensor(10.0, device="cuda"))
    m.kl_hash_interior(g, x, h[1:2])
    assert h[0].item() != h[1].item()
