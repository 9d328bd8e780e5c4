"""Host model of every global address the LDS z-march tiles load and store
(no GPU).  The tiles load unconditionally, from clamped addresses, so that
the compiler counts the loads in flight exactly; this model restates each
tile's address arithmetic (own rows, halo rows, x-edge and x-halo columns
taken from their periodic images, the level ranges of the prologue and of
the prefetch) over every tile, wave and lane of a grid and checks that each
access lies inside the field's allocation [0, alloc).  The persistent
batched and served forms run the same tile functions on tile lists of the
same (tx, ty, tz) ranges, so they are covered too.

Shapes: small and ragged grids (one lane, one row, one level per tile, rows
narrower than a wave segment), both ghost widths, the library's padded
layouts and the unpadded one, and every vector width, tile height and
z-march length the registry builds."""
import itertools

import numpy as np
import pytest

from paper_2303_12374_amd import inputs, kl

LANES = np.arange(64)


def layouts(itot, jtot, ktot, dtype, gc):
    out = [kl.kl_layout_gc(itot, jtot, ktot, dtype, gc)]
    out.append(inputs.plain_layout(itot, jtot, ktot, gh=gc))
    return out


def eligible(vx, itot, off, js, ks):
    return itot % vx == 0 and (off + 1) % vx == 0 and js % vx == 0 and ks % vx == 0


def wrap_x(c, itot):
    return (c - 1) % itot + 1


class Span:
    """Running min / max of element indices."""

    def __init__(self):
        self.lo, self.hi = np.iinfo(np.int64).max, np.iinfo(np.int64).min

    def add(self, base, lmin, lmax, ks, width=1):
        base = np.asarray(base, np.int64)
        self.lo = min(self.lo, int(base.min()) + lmin * ks)
        self.hi = max(self.hi, int(base.max()) + lmax * ks + width - 1)


def tiles(itot, jtot, ktot, vx, by, kb):
    tw = 64 * vx
    nbx, nby, nbz = -(-itot // tw), -(-jtot // by), -(-ktot // kb)
    return itertools.product(range(nbx), range(nby), range(nbz))


def zl_geometry(itot, jtot, ktot, vx, by, kb, tx, ty, tz, off, js):
    """ZlTile and the address bases shared by the zl, step and pair tiles,
    arrays over (wave r, lane)."""
    r = np.arange(by)[:, None]
    lane = LANES[None, :]
    i0w = 1 + tx * 64 * vx
    j0 = 1 + ty * by
    nv = min(by, jtot - j0 + 1)
    k0 = 1 + tz * kb
    k1 = min(k0 + kb, ktot + 1)
    nlanes = min(64, (itot - i0w + 1) // vx)
    top = nv if nv < by else by - 1
    xrow_g = np.where(r == 0, j0 - 1, np.where(r == top, j0 + nv, -1))
    xl = itot - 1 if i0w == 1 else -1
    xr = 1 - i0w if i0w + nlanes * vx > itot else nlanes * vx
    lane_c = np.minimum(lane, nlanes - 1)
    row_c = off + i0w + np.minimum(j0 + r, jtot) * js
    c_own = row_c + lane_c * vx
    c_x = np.where(xrow_g >= 0, off + i0w + lane_c * vx + xrow_g * js, c_own)
    le = max(nlanes - 1, 1)
    c_e = np.where(lane == 0, row_c + xl, np.where(lane == le, row_c + xr, c_own))
    x_is_top = (xrow_g >= 0) & (np.broadcast_to(xrow_g, (by, 1)) == j0 + nv) & (r > 0)
    xrow0 = off + i0w + np.maximum(xrow_g, 0) * js
    return dict(i0w=i0w, j0=j0, nv=nv, k0=k0, k1=k1, nlanes=nlanes, lane=lane, r=r, row_c=row_c, c_own=c_own,
                c_x=c_x, c_e=c_e, le=le, xl=xl, xr=xr, xrow_g=xrow_g, xrow0=xrow0, x_is_top=x_is_top,
                lane_c=lane_c)


def span_diff(g, vx, ks, sp):
    k0, k1 = g["k0"], g["k1"]
    sp.add(g["c_own"], k0 - 1, max(k0 + 1, k1), ks, vx)   # field ring (prologue k0-1 .. k0+2, prefetch <= k1)
    sp.add(g["c_own"], k0, k1, ks, vx)                    # tendencies (own level, then k+1 <= k1)
    sp.add(g["c_x"], k0, k1, ks, vx)                      # halo row (or a re-read of the own row)
    sp.add(g["c_e"], k0, k1, ks)                          # x edges


def span_advec(g, vx, ks, sp):
    k0, k1 = g["k0"], g["k1"]
    lane, xl, x_is_top, xrow0, row_c = g["lane"], g["xl"], g["x_is_top"], g["xrow0"], g["row_c"]
    sp.add(g["c_own"], k0 - 1, max(k0 + 1, k1), ks, vx)   # u ring
    sp.add(g["c_own"], k0, max(k0 + 1, k1), ks, vx)       # w ring, v, ut
    sp.add(g["c_x"], k0, k1, ks, vx)                      # u and v halo rows
    sp.add(g["c_e"], k0, k1, ks)                          # u edges
    c_ev = np.where(lane == 0, row_c + xl, np.where((lane == 1) & x_is_top, xrow0 + xl, g["c_own"]))
    sp.add(c_ev, k0, k1, ks)
    c_ew = np.where(lane == 0, row_c + xl, g["c_own"])
    sp.add(c_ew, k0, max(k0 + 1, k1), ks)


def span_step(g, vx, ks, sp, mode_pair, itot, jtot, ktot, off, js):
    k0, k1 = g["k0"], g["k1"]
    lane, xl, x_is_top, xrow0 = g["lane"], g["xl"], g["x_is_top"], g["xrow0"]
    sp.add(g["c_own"], k0 - 1, max(k0 + 1, k1), ks, vx)
    sp.add(g["c_x"], k0, k1, ks, vx)
    sp.add(g["c_e"], k0, max(min(k0 + 2, k1), k1), ks)
    c_xv = np.where(x_is_top & (lane == 0), xrow0 + xl, g["c_own"])
    sp.add(c_xv, k0, k1, ks)
    if mode_pair:
        sp.add(g["c_own"], k0, k1, ks, vx)                # tendencies
        return
    # outputs with their ghost images: rows j, 0, jtot+1; levels k, 0, 1, ktot+1;
    # x ghosts 0 and itot+1 of the first and last segments
    own = (g["r"] < g["nv"]) & (lane < g["nlanes"])
    if not own.any():
        return
    i0 = g["i0w"] + lane * vx
    for yj in (np.minimum(g["j0"] + g["r"], jtot), 0, jtot + 1):
        base = off + np.where(own, i0 + yj * js, off * 0 + 1 + js)  # inactive lanes store nothing
        sp.add(base, 0, ktot + 1, ks, vx)
        sp.add(off + np.zeros_like(base) + yj * js, 0, ktot + 1, ks)           # x ghost 0
        sp.add(off + itot + 1 + np.zeros_like(base) + yj * js, 0, ktot + 1, ks)  # x ghost itot+1


def check(sp, alloc, what):
    assert sp.lo >= 0, f"{what}: access below the allocation (index {sp.lo})"
    assert sp.hi < alloc, f"{what}: access beyond the allocation (index {sp.hi} >= {alloc})"


SHAPES = [(1, 1, 2), (2, 3, 2), (5, 4, 6), (33, 7, 5), (64, 8, 3), (65, 4, 7), (96, 20, 33), (130, 5, 11),
          (256, 3, 70), (260, 6, 9), (192, 64, 64), (512, 9, 40), (40, 24, 6)]
ZL_TILES = [(vx, by, kb) for vx in (1, 2, 4) for by in (2, 4, 8, 16) for kb in (8, 16, 32, 64, 128, 256, 512)]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_zl_step_and_pair_tiles_stay_inside_the_fields(shape, dtype):
    itot, jtot, ktot = shape
    ran = 0
    for gc in (1, 3):
        for off, js, ks, alloc in layouts(itot, jtot, ktot, dtype, gc):
            for vx, by, kb in ZL_TILES:
                if not eligible(vx, itot, off, js, ks) or (dtype == 1 and vx == 4):
                    continue
                sp_d, sp_a, sp_s, sp_p = Span(), Span(), Span(), Span()
                for tx, ty, tz in tiles(itot, jtot, ktot, vx, by, kb):
                    g = zl_geometry(itot, jtot, ktot, vx, by, kb, tx, ty, tz, off, js)
                    span_diff(g, vx, ks, sp_d)
                    span_advec(g, vx, ks, sp_a)
                    span_step(g, vx, ks, sp_s, False, itot, jtot, ktot, off, js)
                    span_step(g, vx, ks, sp_p, True, itot, jtot, ktot, off, js)
                what = f"{shape} gc={gc} layout=({off},{js},{ks}) vx={vx} by={by} kb={kb}"
                for name, sp in (("diff_uvw", sp_d), ("advec_u", sp_a), ("step", sp_s), ("advec_diff", sp_p)):
                    check(sp, alloc, f"{name} {what}")
                ran += 1
    assert ran > 0


def a5_spans(itot, jtot, ktot, vx, by, kb, off, js, ks, pair):
    """advec_u_2i5 tiles (a5 / a5s: pair = False; a5p: pair = True)."""
    sp = Span()
    nh = (6 + by - 1) // by
    r = np.arange(by)[:, None]
    lane = LANES[None, :]
    for tx, ty, tz in tiles(itot, jtot, ktot, vx, by, kb):
        i0w = 1 + tx * 64 * vx
        nlanes = min(64, (itot - i0w + 1) // vx)
        j0 = 1 + ty * by
        nv = min(by, jtot - j0 + 1)
        k0 = 1 + tz * kb
        k1 = min(k0 + kb, ktot + 1)
        lane_c = np.minimum(lane, nlanes - 1)
        if not pair:
            rowo = off + i0w + np.minimum(j0 + r, jtot) * js
            c_own = rowo + lane_c * vx
            ecol = np.where(lane < 3, wrap_x(i0w - 3 + lane, itot) - i0w,
                            np.where(lane < 6, wrap_x(i0w + nlanes * vx + lane - 3, itot) - i0w, lane_c * vx))
            e_own = rowo + ecol
            xl1 = wrap_x(i0w - 1, itot) - i0w
            hcs, hes = [], []
            for m in range(nh):
                h = r + m * by
                hrho = np.where(h < 6, np.where(h < 3, h, nv + h), -1)
                hrow0 = off + i0w + (j0 - 3 + np.where(hrho < 0, 3, hrho)) * js
                hcs.append(np.where(hrho < 0, c_own, hrow0 + lane_c * vx))
                hes.append(np.where(hrho < 0, c_own, hrow0 + ecol))
            vhalo = r == by - 1
            vrow = off + i0w + (j0 + nv) * js
            c_vh = np.where(vhalo, vrow + lane_c * vx, c_own)
            e_v = np.where(lane == 0, rowo + xl1, np.where((lane == 1) & vhalo, vrow + xl1, c_own))
            e_w = np.where(lane == 0, rowo + xl1, c_own)
            # u window by guarded column loads (levels clipped to [0, ktot+1])
            sp.add(c_own, max(k0 - 3, 0), min(k1 + 3, ktot + 1), ks, vx)
            lmax = k1 - 1
            for b in hcs:
                sp.add(b, k0, lmax, ks, vx)
            for b in hes:
                sp.add(b, k0, lmax, ks)
            sp.add(e_own, k0, lmax, ks)
            sp.add(c_own, k0, lmax + 1, ks, vx)        # v own row, w at k+1, ut
            sp.add(c_vh, k0, lmax, ks, vx)
            sp.add(e_v, k0, lmax, ks)
            sp.add(e_w, k0, lmax + 1, ks)
        else:
            own = r < nv
            on = lane < nlanes
            row0 = off + i0w + lane * vx
            c_own = row0 + (j0 + r) * js
            e_own = off + i0w + (j0 + r) * js
            iend = i0w + nlanes * vx - 1
            xlo = [wrap_x(i0w - 3 + e, itot) - i0w for e in range(3)]
            xhi = [wrap_x(iend + 1 + e, itot) - i0w for e in range(3)]
            mask = own & on
            if mask.any():
                sp.add(c_own[mask], max(k0 - 3, 0), min(k1 + 6, ktot + 1), ks, vx)
                sp.add(c_own[mask], k0, k1, ks, vx)
            if own.any():
                eo = np.broadcast_to(e_own, (by, 1))[own[:, 0]]
                for o in xlo + xhi:
                    sp.add(eo + o, k0, k1, ks)
            for m in range(nh):
                h = r + m * by
                hrho = np.where(h < 6, np.where(h < 3, h, nv + h), -1)
                jg = j0 - 3 + np.where(hrho < 0, 3, hrho)
                hon = (hrho >= 0)[:, 0]
                if hon.any():
                    hc = (row0 + jg * js)[hon][:, :nlanes]
                    he = (off + i0w + jg * js)[hon]
                    sp.add(hc, k0, k1, ks, vx)
                    for o in xlo + xhi:
                        sp.add(he + o, k0, k1, ks)
            c_vh = off + i0w + lane[:, :nlanes] * vx + (j0 + nv) * js
            sp.add(c_vh, k0, k1, ks, vx)
            sp.add(np.array([off + i0w + (j0 + nv) * js + xlo[2]]), k0, k1, ks)
    return sp


def a5r_spans(itot, jtot, ktot, vx, by, kb, off, js, ks, esize):
    """advec_u_2i5 parity-slot tiles (a5r): a uniform base per level (i = 1,
    j = j0 - 3) plus unsigned 32-bit per-lane byte offsets, which must be
    non-negative and below 2^32."""
    sp = Span()
    nh = (6 + by - 1) // by
    r = np.arange(by)[:, None]
    lane = LANES[None, :]
    for tx, ty, tz in tiles(itot, jtot, ktot, vx, by, kb):
        i0w = 1 + tx * 64 * vx
        nlanes = min(64, (itot - i0w + 1) // vx)
        j0 = 1 + ty * by
        nv = min(by, jtot - j0 + 1)
        k0 = 1 + tz * kb
        k1 = min(k0 + kb, ktot + 1)
        tb = off + 1 + (j0 - 3) * js
        lane_c = np.minimum(lane, nlanes - 1)
        rown = 3 + np.minimum(r, jtot - j0)
        cx = i0w - 1 + lane_c * vx
        o_own = rown * js + cx
        ecol = np.where(lane < 3, wrap_x(i0w - 3 + lane, itot) - 1,
                        np.where(lane < 6, wrap_x(i0w + nlanes * vx + lane - 3, itot) - 1, cx))
        o_eown = rown * js + ecol
        xl1 = wrap_x(i0w - 1, itot) - 1
        o_hc, o_he = [], []
        for m in range(nh):
            h = r + m * by
            rho = np.where(h < 6, np.where(h < 3, h, nv + h), -1)
            o_hc.append(np.where(rho >= 0, rho * js + cx, o_own))
            o_he.append(np.where(rho >= 0, rho * js + ecol, o_own))
        vhalo = r == by - 1
        vrel = 3 + nv
        o_vh = np.where(vhalo, vrel * js + cx, o_own)
        o_ev = np.where(lane == 0, rown * js + xl1, np.where((lane == 1) & vhalo, vrel * js + xl1, o_own))
        o_ew = np.where(lane == 0, rown * js + xl1, o_own)
        for o in [o_own, o_eown, o_vh, o_ev, o_ew] + o_hc + o_he:
            o = np.broadcast_to(o, (by, 64))
            assert o.min() >= 0 and (o.max() + vx) * esize < 2 ** 32, "a5r offset outside [0, 2^32)"
        lo, hi = k0, k1 - 1  # levels of load_level and of the ut store
        top = lambda k: min(k, ktot + 1)
        sp.add(tb + o_own, max(k0 - 3, 0), top(k0 + 3), ks, vx)   # window and face k0's bottom value
        sp.add(tb + o_own, top(k0 + 4), top(hi + 5), ks, vx)      # window tops
        sp.add(tb + o_own, k0, hi + 1, ks, vx)                    # own v row, w one level up, ut
        sp.add(tb + o_ew, k0, hi + 1, ks)                          # w's left neighbour (face k0: level k0)
        for o in o_hc:
            sp.add(tb + o, lo, hi, ks, vx)
        for o in o_he:
            sp.add(tb + o, lo, hi, ks)
        sp.add(tb + o_eown, lo, hi, ks)
        sp.add(tb + o_vh, lo, hi, ks, vx)
        sp.add(tb + o_ev, lo, hi, ks)
    return sp


def s2_spans(itot, jtot, ktot, vx, by, kb, off, js, ks):
    """diff_smag tiles: rows from a wave-uniform row start (column 0) plus a
    per-lane offset.  The parity-slot tile (s2r) loads the same rows over
    the same levels (its prefetch of level k+3 is clamped to k1 as the
    s2 tile's of level k+2), so this span covers both."""
    sp = Span()
    nh = (8 + by - 1) // by
    r = np.arange(by)[:, None]
    lane = LANES[None, :]
    for tx, ty, tz in tiles(itot, jtot, ktot, vx, by, kb):
        i0w = 1 + tx * 64 * vx
        nlanes = min(64, (itot - i0w + 1) // vx)
        j0 = 1 + ty * by
        nv = min(by, jtot - j0 + 1)
        k0 = 1 + tz * kb
        k1 = min(k0 + kb, ktot + 1)
        lane_c = np.minimum(lane, nlanes - 1)
        le = max(nlanes - 1, 1)
        row_c = off + np.minimum(j0 + r, jtot) * js
        o_pt = i0w + lane_c * vx
        o_e = np.where(lane == 0, wrap_x(i0w - 1, itot), np.where(lane == le, wrap_x(i0w + nlanes * vx, itot), o_pt))
        sp.add(row_c + o_pt, k0 - 1, k1, ks, vx)        # load_plane levels k0-1 .. min(k+2, k1); tendencies
        sp.add(row_c + o_e, k0 - 1, k1, ks)
        for m in range(nh):
            h = r + m * by
            hf = np.where(h < 8, h >> 1, -1)
            hrow = np.where(h & 1, nv + 1, 0)
            hr0 = np.where(hf < 0, row_c, off + (j0 - 1 + hrow) * js)
            sp.add(hr0 + o_pt, k0 - 1, k1, ks, vx)
            sp.add(hr0 + o_e, k0 - 1, k1, ks)
    return sp


A5_TILES = [(vx, by, kb) for vx in (1, 2, 4) for by in (2, 4, 8, 16) for kb in (16, 32, 64, 128, 256)]
LES_SHAPES = [(1, 1, 2), (2, 3, 2), (4, 3, 5), (5, 4, 6), (33, 7, 5), (64, 8, 3), (65, 4, 7), (130, 5, 11),
              (256, 3, 70), (260, 6, 9), (40, 24, 6)]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("shape", LES_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_les_tiles_stay_inside_the_fields(shape, dtype):
    itot, jtot, ktot = shape
    ran = 0
    for off, js, ks, alloc in layouts(itot, jtot, ktot, dtype, 3):
        for vx, by, kb in A5_TILES:
            if not eligible(vx, itot, off, js, ks) or (dtype == 1 and vx == 4):
                continue
            what = f"{shape} layout=({off},{js},{ks}) vx={vx} by={by} kb={kb}"
            check(a5_spans(itot, jtot, ktot, vx, by, kb, off, js, ks, False), alloc, f"a5 {what}")
            check(a5_spans(itot, jtot, ktot, vx, by, kb, off, js, ks, True), alloc, f"a5p {what}")
            check(a5r_spans(itot, jtot, ktot, vx, by, kb, off, js, ks, 4 if dtype == 0 else 8), alloc,
                  f"a5r {what}")
            check(s2_spans(itot, jtot, ktot, vx, by, kb, off, js, ks), alloc, f"s2 {what}")
            ran += 1
    assert ran > 0


def test_model_catches_an_out_of_bounds_halo():
    """The model is not vacuous: a tile whose top halo row were taken one row
    further (j0 + nv + 1, past the ghost row) leaves the allocation of the
    unpadded layout of a grid whose last tile reaches the top."""
    itot, jtot, ktot = 64, 8, 4
    off, js, ks, alloc = inputs.plain_layout(itot, jtot, ktot)
    sp = Span()
    for tx, ty, tz in tiles(itot, jtot, ktot, 1, 8, 8):
        g = zl_geometry(itot, jtot, ktot, 1, 8, 8, tx, ty, tz, off, js)
        bad = np.where(g["xrow_g"] >= 0, g["c_x"] + js * (g["xrow_g"] == g["j0"] + g["nv"]), g["c_own"])
        sp.add(bad, g["k0"], g["k1"], ks)
    with pytest.raises(AssertionError):
        check(sp, alloc, "planted")
