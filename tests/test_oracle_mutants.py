"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Every mutant is a one-token edit of ``oracle/oracle.c`` (a dropped term, a
wrong sign, a wrong index, a transposed operand), compiled on the CPU into a
temporary library; the pins of ``pins.py`` are then run against it.
"""
import os

import pytest

import oracle
import pins

# (name, function the edit lands in, original text, mutated text)
MUTANTS = [
    ("advec_dzi_index", "advec_u_at", "* dzi[k];", "* dzi[k + 1];"),
    ("advec_y_sign", "advec_u_at", "vn * un - vs * us", "vn * un + vs * us"),
    ("advec_v_xoffset", "advec_u_at", "interp(v[at(g, i - 1, j + 1, k)]", "interp(v[at(g, i + 1, j + 1, k)]"),
    ("advec_drop_y", "advec_u_at", "-(adv_x + adv_y + adv_z)", "-(adv_x + adv_z)"),
    ("advec_transposed_x", "advec_u_at", "fx_hi * fx_hi - fx_lo * fx_lo", "fx_lo * fx_lo - fx_hi * fx_hi"),
    ("advec_w_level", "advec_u_at", "interp(w[at(g, i - 1, j, k)], w[at(g, i, j, k)])",
     "interp(w[at(g, i - 1, j, k + 1)], w[at(g, i, j, k)])"),
    ("advec_u_zinterp", "advec_u_at", "interp(u[at(g, i, j, k - 1)], uc)", "interp(u[at(g, i, j, k + 1)], uc)"),
    ("diff_dzhi_index", "diff_c_at", "* dzhi[k + 1]", "* dzhi[k]"),
    ("diff_w_dzi_index", "diff_w_at", "* dzi[k - 1]) * dzhi[k]", "* dzi[k]) * dzhi[k]"),
    ("diff_dxi_square", "ora_diff_uvw", "dxi2 = dxi * dxi", "dxi2 = dxi"),
    ("diff_lap_sign", "lap_xy", "- 2.0 * c + f[at(g, i - 1, j, k)]", "+ 2.0 * c + f[at(g, i - 1, j, k)]"),
    ("diff_w_range", "ora_diff_uvw", "if (k >= kw0)\n                    wt[c]", "if (k >= 1)\n                    wt[c]"),
    ("fill_x_source", "fill_xy", "f[at(g, 0, j, k)] = f[at(g, g->itot, j, k)]", "f[at(g, 0, j, k)] = f[at(g, 1, j, k)]"),
    ("fill_w_nopen_sign", "ora_fill_ghosts", "copy_plane(&g, w, 0, 2, -1.0);", "copy_plane(&g, w, 0, 2, 1.0);"),
    ("fill_periodic_z", "ora_fill_ghosts", "copy_plane(&g, f3[n], 0, kt, 1.0);", "copy_plane(&g, f3[n], 0, 1, 1.0);"),
    ("fill_w_top", "ora_fill_ghosts", "copy_plane(&g, w, kt + 1, kt, 1.0);\n        copy_plane(&g, w, 0, 2",
     "copy_plane(&g, w, kt + 1, kt - 1, 1.0);\n        copy_plane(&g, w, 0, 2"),
    ("euler_wrong_tendency", "ora_euler", "u[c] += dt * ut[c];", "u[c] += dt * vt[c];"),
    ("conservation_weight", "ora_conservation", "s2 += wt[c] * (1.0 / dzhi[k])", "s2 += wt[c] * (1.0 / dzi[k])"),
    ("checksum_square", "ora_checksums", "s2 += x * x;", "s2 += x;"),
]


@pytest.mark.parametrize("name,fn,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, fn, orig, mut, tmp_path):
    src = open(oracle.SRC).read()
    start = src.index(f" {fn}(")
    start = src.index("{", start)
    end = src.index("\n}\n", start)
    body = src[start:end]
    assert body.count(orig) == 1, f"mutation anchor for {name} must occur once in {fn}"
    path = tmp_path / f"{name}.c"
    path.write_text(src[:start] + body.replace(orig, mut) + src[end:])
    so = str(tmp_path / f"lib{name}.so")
    oracle.build(str(path), so, openmp=False)
    lib = oracle.load(so)
    failed = []
    for pin in pins.PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} survived every pin"
