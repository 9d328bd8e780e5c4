"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Every mutant is a one-token edit of ``oracle/oracle.c`` (a dropped term, a
wrong sign, a wrong index, a transposed operand), compiled on the CPU into a
temporary library; the pins of ``pins.py`` are then run against it.
"""
import os

import pytest

import oracle
import pins
import pins_les

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
    ("fill_x_source", "fill_xy", "f[at(g, 1 - m, j, k)] = f[at(g, wrap(1 - m, g->itot), j, k)]",
     "f[at(g, 1 - m, j, k)] = f[at(g, wrap(2 - m, g->itot), j, k)]"),
    ("fill_y_far_ghost", "fill_xy", "f[at(g, i, g->jtot + m, k)] = f[at(g, i, wrap(g->jtot + m, g->jtot), k)]",
     "f[at(g, i, g->jtot + m, k)] = f[at(g, i, wrap(g->jtot + 1, g->jtot), k)]"),
    ("fill_w_nopen_sign", "fill_all", "copy_plane(g, w, 0, 2, -1.0);", "copy_plane(g, w, 0, 2, 1.0);"),
    ("fill_periodic_z", "fill_all", "copy_plane(g, f3[n], 0, kt, 1.0);", "copy_plane(g, f3[n], 0, 1, 1.0);"),
    ("fill_w_top", "fill_all", "copy_plane(g, w, kt + 1, kt, 1.0);\n        copy_plane(g, w, 0, 2",
     "copy_plane(g, w, kt + 1, kt - 1, 1.0);\n        copy_plane(g, w, 0, 2"),
    ("euler_wrong_tendency", "ora_euler", "u[c] += dt * ut[c];", "u[c] += dt * vt[c];"),
    ("conservation_weight", "ora_conservation", "s2 += wt[c] * (1.0 / dzhi[k])", "s2 += wt[c] * (1.0 / dzi[k])"),
    ("checksum_square", "ora_checksums", "s2 += x * x;", "s2 += x;"),
    # fifth-order advection
    ("c6_coefficient", "flux5", "37.0 * (a0 + a1) - 8.0", "36.0 * (a0 + a1) - 8.0"),
    ("c6_outer_pair", "flux5", "+ (am2 + a3)) / 60.0", "+ (am1 + a3)) / 60.0"),
    ("d5_sign", "flux5", "return U * c6 - fabs(U) * d5;", "return U * c6 + fabs(U) * d5;"),
    ("d5_middle", "flux5", "- 5.0 * (a2 - am1)", "- 5.0 * (a2 - a0)"),
    ("d3_sign", "flux3", "return U * c4 - fabs(U) * d3;", "return U * c4 + fabs(U) * d3;"),
    ("c4_weights", "flux3", "(7.0 * (a0 + a1) - (am1 + a2)) / 12.0", "(7.0 * (a0 + a1) - (am1 + a2)) / 13.0"),
    ("ladder_third", "flux_z_2i5", "if (kf == 2 || kf == g->ktot)", "if (kf == 2)"),
    ("ladder_second", "flux_z_2i5", "if (kf == 1 || kf == g->ktot + 1)", "if (kf == 1)"),
    ("z_w_level", "flux_z_2i5", "interp(w[at(g, i - 1, j, kf)], w[at(g, i, j, kf)])",
     "interp(w[at(g, i - 1, j, kf - 1)], w[at(g, i, j, kf)])"),
    ("x5_stencil_shift", "advec_u_2i5_at", "fw = flux5(Uw, u[at(g, i - 3, j, k)]", "fw = flux5(Uw, u[at(g, i - 2, j, k)]"),
    ("y5_v_offset", "advec_u_2i5_at", "Vn = interp(v[at(g, i - 1, j + 1, k)]", "Vn = interp(v[at(g, i + 1, j + 1, k)]"),
    ("y5_far_point", "advec_u_2i5_at", "u[at(g, i, j + 2, k)], u[at(g, i, j + 3, k)]);",
     "u[at(g, i, j + 2, k)], u[at(g, i, j + 2, k)]);"),
    ("adv5_drop_z", "advec_u_2i5_at", "-(adv_x + adv_y + adv_z)", "-(adv_x + adv_y)"),
    # stress-divergence diffusion
    ("smag_u_normal_factor", "smag_u_at", "(2.0 * dxi * dxi)", "(dxi * dxi)"),
    ("smag_u_edge_mean", "smag_u_at", "e[at(g, i - 1, j + 1, k)], e[at(g, i, j + 1, k)]);",
     "e[at(g, i - 1, j + 1, k)], e[at(g, i + 1, j + 1, k)]);"),
    ("smag_u_cross_v", "smag_u_at", "(v[at(g, i, j + 1, k)] - v[at(g, i - 1, j + 1, k)]) * dxi",
     "(v[at(g, i, j + 1, k)] - v[at(g, i - 1, j, k)]) * dxi"),
    ("smag_u_cross_w_metric", "smag_u_at", "(w[at(g, i, j, k)] - w[at(g, i - 1, j, k)]) * dxi)) * dzi[k]",
     "(w[at(g, i, j, k)] - w[at(g, i - 1, j, k)]) * dyi)) * dzi[k]"),
    ("smag_v_edge_mean", "smag_v_at", "ee = mean4(e[at(g, i, j - 1, k)], e[at(g, i + 1, j - 1, k)]",
     "ee = mean4(e[at(g, i, j - 1, k)], e[at(g, i - 1, j - 1, k)]"),
    ("smag_v_cross_u", "smag_v_at", "(u[at(g, i + 1, j, k)] - u[at(g, i + 1, j - 1, k)]) * dyi",
     "(u[at(g, i + 1, j, k)] - u[at(g, i, j - 1, k)]) * dyi"),
    ("smag_w_zz_metric", "smag_w_at", "(wc - w[at(g, i, j, k - 1)]) * dzi[k - 1])", "(wc - w[at(g, i, j, k - 1)]) * dzi[k])"),
    ("smag_w_cross_dzhi", "smag_w_at", "(v[at(g, i, j + 1, k)] - v[at(g, i, j + 1, k - 1)]) * dzhi[k])",
     "(v[at(g, i, j + 1, k)] - v[at(g, i, j + 1, k - 1)]) * dzhi[k + 1])"),
    ("smag_w_range", "ora_diff_smag", "if (k >= kw0)\n                    wt[c] += smag_w_at",
     "if (k >= 1)\n                    wt[c] += smag_w_at"),
    ("smag_mean4", "mean4", "0.25 * (a + b + c + d)", "0.25 * (a + b + c + c)"),
    ("fill_scalar_wall", "ora_fill_scalar", "copy_plane(&g, f, ktot + 1, ktot, 1.0);", "copy_plane(&g, f, ktot + 1, 1, 1.0);"),
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
    for pin in pins.PINS + pins_les.PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} survived every pin"
