"""Served form: continuous batching of stencil-step requests.  Each result
matches the CPU oracle, is bitwise the same alone and in a mix, and
admission respects the memory budget."""
import json
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2303_12374_amd import inputs
from gpu_util import TOL, rel_err

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


class Server:
    def __init__(self, arena_bytes=1 << 30, budget=None):
        m = kl()
        self.m = m
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        self.h = m.kl_server_create(self.arena, arena_bytes, budget or arena_bytes)

    def wait(self, ticket, timeout=60.0):
        t0 = time.time()
        while True:
            rc, res = self.m.kl_poll(self.h, ticket)
            if rc == self.m.OK:
                return res
            if time.time() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done")
            time.sleep(0.001)

    def fields(self, res, req):
        """Host copies (ktot+2, jtot+2, itot+2) of the result's u, v, w."""
        itot, jtot, ktot, dtype = req[:4]
        tdt = self.m.TORCH_DTYPE[dtype]
        s = 4 if dtype == 0 else 8
        out = []
        for n in range(3):
            start = res.fields[n] - self.arena.data_ptr()
            nelem = res.off + res.kstride * (ktot + 2)
            flat = self.arena[start:start + nelem * s].view(tdt)
            box = flat.as_strided((ktot + 2, jtot + 2, itot + 2), (res.kstride, res.jstride, 1),
                                  flat.storage_offset() + res.off)
            out.append(box.cpu().numpy().astype(np.float64))
        return out

    def close(self):
        self.m.kl_server_destroy(self.h)


def oracle_run(itot, jtot, ktot, dtype, bc, nsteps, dt, visc, seed):
    """The oracle's state after nsteps steps from the served initial state."""
    npd = np.float32 if dtype == 0 else np.float64
    Lz = inputs.domain_height(itot, jtot, ktot)
    zg = inputs.zgrid(ktot, Lz, 0.0 if bc == 2 else 1.5)
    off, js, ks, alloc = inputs.plain_layout(itot, jtot, ktot)
    g = oracle.Grid(itot, jtot, ktot, off, js, ks, alloc, float(npd(itot)), float(npd(jtot)),
                    zg["dzi"].astype(npd).astype(np.float64), zg["dzhi"].astype(npd).astype(np.float64), bc)
    fs = [f.astype(npd).astype(np.float64) for f in inputs.random_fields(seed, itot, jtot, ktot)]
    host = [inputs.embed(f, off, js, ks, alloc) for f in fs]
    oracle.fill_ghosts(g, *host)
    tmp = [np.zeros(alloc) for _ in range(3)]
    for _ in range(nsteps):
        oracle.step(g, float(npd(visc)), float(npd(dt)), *host, *tmp)
        if dtype == 0:
            host = [h.astype(np.float32).astype(np.float64) for h in host]
    return [inputs.padded_view(h, itot, jtot, ktot, off, js, ks).copy() for h in host], g, host


@pytest.mark.parametrize("dtype,bc", [(0, 0), (1, 0), (1, 2), (0, 1)])
def test_served_request_matches_oracle(dtype, bc):
    S = Server()
    try:
        req = (40, 24, 16, dtype, bc, 3, 2e-3, 1e-5, 77)
        t = S.m.kl_submit(S.h, *req)
        res = S.wait(t)
        assert res.state == 2 and res.err == 0
        assert res.t_arrive_ns <= res.t_admit_ns <= res.t_done_ns
        got = S.fields(res, req)
        ref, g, host = oracle_run(*req[:3], dtype, bc, 3, 2e-3, 1e-5, 77)
        # 3 steps: the state error stays far inside the kernel tolerance (the
        # derivation is in test_gpu_parity.test_step_matches_oracle)
        for a, b in zip(got, ref):
            assert rel_err(a, b) <= TOL[dtype]
        # FP64 checksums of the final state
        cs = np.array(res.checksum)
        for n in range(3):
            x = b = ref[n][1:-1, 1:-1, 1:-1]
            assert abs(cs[3 * n] - np.sum(x)) <= 1e-6 * np.sum(np.abs(x)) + 1e-9
            assert abs(cs[3 * n + 2] - np.max(np.abs(x))) <= 1e-5 * np.max(np.abs(x))
        S.m.kl_release(S.h, t)
    finally:
        S.close()


def test_alone_and_in_a_mix_are_bitwise_equal():
    S = Server(arena_bytes=3 << 30)
    try:
        probe = (64, 48, 20, 0, 0, 4, 1e-3, 1e-5, 5)
        t = S.m.kl_submit(S.h, *probe)
        alone = S.fields(S.wait(t), probe)
        S.m.kl_release(S.h, t)
        rng = np.random.default_rng(0)
        mix = []
        for n in range(14):
            shape = [int(x) for x in rng.choice([16, 32, 48, 64, 96], 3)]
            shape[2] = max(shape[2], 2)
            mix.append((*shape, int(rng.integers(0, 2)), int(rng.integers(0, 3)), int(rng.integers(1, 6)),
                        1e-3, 1e-5, 100 + n))
        tickets = []
        for n, r in enumerate(mix):
            tickets.append((S.m.kl_submit(S.h, *r), r))
            if n == 6:
                tickets.append((S.m.kl_submit(S.h, *probe), probe))
        results = {tk: S.wait(tk) for tk, _ in tickets}
        for tk, r in tickets:
            if r == probe:
                got = S.fields(results[tk], r)
                for a, b in zip(got, alone):
                    assert np.array_equal(a, b), "served result changed with its neighbours"
        st = S.m.kl_server_stats(S.h)
        assert st[2] == len(tickets) + 1
        for tk, _ in tickets:
            S.m.kl_release(S.h, tk)
    finally:
        S.close()


def test_sixty_request_mix_equals_each_request_alone():
    """Every request of a 60-request mix (both precisions, all boundary
    modes, ragged shapes, 1-6 steps) equals, bitwise, the same request served
    on its own; the FP64 checksums agree bitwise too."""
    S = Server(arena_bytes=3 << 30)
    try:
        rng = np.random.default_rng(11)
        mix = []
        for n in range(60):
            shape = [int(x) for x in rng.choice([8, 16, 24, 33, 48, 64, 72], 3)]
            shape[2] = max(shape[2], 2)
            mix.append((*shape, int(rng.integers(0, 2)), int(rng.integers(0, 3)), int(rng.integers(1, 7)),
                        1e-3, 1e-5, 500 + n))
        tickets = [S.m.kl_submit(S.h, *r) for r in mix]
        in_mix = {}
        for tk, r in zip(tickets, mix):
            res = S.wait(tk)
            in_mix[tk] = (S.fields(res, r), list(res.checksum))
            S.m.kl_release(S.h, tk)
        for tk, r in zip(tickets, mix):
            t = S.m.kl_submit(S.h, *r)
            res = S.wait(t)
            alone = S.fields(res, r)
            for a, b in zip(in_mix[tk][0], alone):
                assert np.array_equal(a, b), f"request {r} differs alone and in the mix"
            assert list(res.checksum) == in_mix[tk][1], f"request {r}: checksums differ"
            S.m.kl_release(S.h, t)
    finally:
        S.close()


def test_served_equals_single_grid_steps():
    """A served request equals the same steps run with kl_step on its own grid."""
    m = kl()
    S = Server()
    try:
        req = (48, 32, 12, 1, 2, 3, 1e-3, 1e-5, 9)
        t = S.m.kl_submit(S.h, *req)
        got = S.fields(S.wait(t), req)
    finally:
        S.close()
    g = m.Grid(48, 32, 12, dtype=1, bc=2)
    f = [g.full() for _ in range(3)]
    m.kl_generate_fields(g, 9, *f)
    m.kl_fill_ghosts(g, *f)
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    for _ in range(3):
        m.kl_step(g, 1e-5, 1e-3, *f, *tend)
    for a, b in zip(got, f):
        assert np.array_equal(a, g.box(b).cpu().numpy())


def test_budget_admission_and_errors():
    m = kl()
    small = (32, 32, 16, 0, 0, 2, 1e-3, 1e-5, 1)
    off, js, ks, alloc = m.kl_layout(32, 32, 16, 0)
    one = 6 * ((alloc * 4 + 255) // 256 * 256) + 2 * 256
    S = Server(arena_bytes=64 << 20, budget=int(one * 1.5))
    try:
        with pytest.raises(m.KLError) as e:
            S.m.kl_submit(S.h, 128, 128, 128, 0, 0, 1, 1e-3, 1e-5, 0)
        assert e.value.code == m.ERR_BUDGET
        with pytest.raises(m.KLError) as e:
            S.m.kl_submit(S.h, 0, 8, 8, 0, 0, 1, 1e-3, 1e-5, 0)
        assert e.value.code == m.ERR_INVALID
        tickets = [S.m.kl_submit(S.h, *small) for _ in range(4)]
        done = []
        for tk in tickets:  # only one fits at a time: each runs after the previous is released
            res = S.wait(tk)
            done.append(res)
            S.m.kl_release(S.h, tk)
        st = S.m.kl_server_stats(S.h)
        assert st[3] <= int(one * 1.5), "peak bytes above the budget"
        assert st[2] == 4
        for a, b in zip(done, done[1:]):
            assert b.t_admit_ns >= a.t_done_ns
        with pytest.raises(m.KLError) as e:
            S.m.kl_poll(S.h, 10 ** 9)
        assert e.value.code == m.ERR_NOTFOUND
    finally:
        S.close()


@pytest.mark.parametrize("dtype,shape,bc", [(0, (256, 20, 40), 0), (1, (128, 20, 40), 1)])
def test_every_step_configuration_served_bitwise(tmp_path, dtype, shape, bc):
    """Each fused-step configuration, forced by a wisdom record for the
    request's shape, serves a request (ragged y and z tiles) bitwise equal to
    kl_step on its own grid; a configuration without a persistent form falls
    back to one sized to the grid, which must agree just the same."""
    m = kl()
    itot, jtot, ktot = shape
    nsteps, dt, visc, seed = 2, 1e-3, 1e-5, 21
    g = m.Grid(itot, jtot, ktot, dtype=dtype, bc=bc)
    f = [g.full() for _ in range(3)]
    m.kl_generate_fields(g, seed, *f)
    m.kl_fill_ghosts(g, *f)
    tend = [g.zeros_interior(fill=0.0) for _ in range(3)]
    for _ in range(nsteps):
        m.kl_step(g, visc, dt, *f, *tend)
    ref = [g.box(x).cpu().numpy().astype(np.float64) for x in f]
    wdir = tmp_path / "forced"
    wdir.mkdir()
    req = (itot, jtot, ktot, dtype, bc, nsteps, dt, visc, seed)
    S = Server(arena_bytes=1 << 28)
    served = 0
    try:
        for i in range(m.kl_num_variants(m.STEP, dtype)):
            name = m.kl_variant_name(m.STEP, dtype, i)
            rec = {"kernel": "step", "dtype": "f32" if dtype == 0 else "f64", "problem_size": list(shape),
                   "variant": name, "device": "forced", "arch": "gfx950", "time_ms": 1.0}
            (wdir / "step.wisdom").write_text(json.dumps(rec) + "\n")
            m.kl_set_wisdom_dir(str(wdir))
            if m.kl_selected_variant(g, m.STEP) != i:
                continue  # not eligible for this grid
            t = S.m.kl_submit(S.h, *req)
            got = S.fields(S.wait(t), req)
            S.m.kl_release(S.h, t)
            for n in range(3):
                assert np.array_equal(got[n], ref[n]), f"{name}: field {n} differs from kl_step"
            served += 1
    finally:
        S.close()
    assert served >= 10
