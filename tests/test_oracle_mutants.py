"""Plant plausible mistakes in copies of the oracle source and check that the
pins catch every one (CPU only; the oracle itself is never modified)."""
import os
import subprocess

import pytest

import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "mobius_oracle.c")

# (name, text in the oracle, planted replacement)
MUTANTS = [
    ("wilson_mass_sign", "out[k] = (4.0 - p->M5) * in", "out[k] = (4.0 + p->M5) * in"),
    ("forward_projector", "one_pm_gamma(mu, -sgn, v, w);", "one_pm_gamma(mu, +sgn, v, w);"),
    ("backward_link_not_daggered", "colour_mul(U + ((int64_t)mu * V + xb) * 9, 1,",
     "colour_mul(U + ((int64_t)mu * V + xb) * 9, 0,"),
    ("hop_factor", "out[k] -= 0.5 * ef * w[k];\n        /* backward",
     "out[k] -= 1.0 * ef * w[k];\n        /* backward"),
    ("mu_adjoint_factors_unswapped",
     "const double ef = mu == 3 ? exp(dag ? -p->mu : p->mu) : 1.0;\n"
     "        const double eb = mu == 3 ? exp(dag ? p->mu : -p->mu) : 1.0;",
     "const double ef = mu == 3 ? exp(p->mu) : 1.0;\n"
     "        const double eb = mu == 3 ? exp(-p->mu) : 1.0;"),
    ("mu_on_a_spatial_direction",
     "const double ef = mu == 3 ? exp(dag ? -p->mu : p->mu) : 1.0;\n"
     "        const double eb = mu == 3 ? exp(dag ? p->mu : -p->mu) : 1.0;",
     "const double ef = mu == 2 ? exp(dag ? -p->mu : p->mu) : 1.0;\n"
     "        const double eb = mu == 2 ? exp(dag ? p->mu : -p->mu) : 1.0;"),
    ("wall_mass_sign", "double fp1 = (s == Ls - 1) ? -p->mf : 1.0;\n            double fm1",
     "double fp1 = (s == Ls - 1) ? p->mf : 1.0;\n            double fm1"),
    ("s_coupling_chirality_swapped",
     "chiral_part(in + ((int64_t)sp1 * V + nb[j]) * SITE_DOF, -1, fp1, wb);\n"
     "                chiral_part(in + ((int64_t)sm1 * V + nb[j]) * SITE_DOF, +1, fm1, wb);",
     "chiral_part(in + ((int64_t)sp1 * V + nb[j]) * SITE_DOF, +1, fp1, wb);\n"
     "                chiral_part(in + ((int64_t)sm1 * V + nb[j]) * SITE_DOF, -1, fm1, wb);"),
    ("c5_dropped_in_adjoint", "y[k] = c5_of(p, sm1) * t2[k]", "y[k] = 0.0 * t2[k]"),
    ("m5inv_transpose_swapped", "int transpose = dag ? minus : !minus;",
     "int transpose = dag ? !minus : minus;"),
    ("m5inv_corner_mass", "mu = p->mf * a;", "mu = p->mf;"),
    ("m5inv_power", "sum += pow(-a, s - 1) * b[(s - 1) * stride];",
     "sum += pow(-a, s) * b[(s - 1) * stride];"),
    ("Mminus_sign", "const double Mm = p->c5 * (4.0 - p->M5) - 1.0;",
     "const double Mm = p->c5 * (4.0 - p->M5) + 1.0;"),
    ("schur_sign", "out[k] = in[k] - t2[k];\n    zero_other_parity(p, out, 1);",
     "out[k] = in[k] + t2[k];\n    zero_other_parity(p, out, 1);"),
    ("reconstruct_parity", "orc_hop(p, U, 0, (double *)xo, (double *)t2, 0);       /* D_eo psi_o",
     "orc_hop(p, U, 1, (double *)xo, (double *)t2, 0);       /* D_eo psi_o"),
    ("cgls_beta_sign", "pv[k] = s[k] + beta * pv[k];", "pv[k] = s[k] - beta * pv[k];"),
    ("cgne_alpha_uses_r", "const double alpha = rr / norm2(t, n);",
     "const double alpha = rr / norm2(q, n);"),
    ("force_imaginary_direction_sign", "E[lid * 9 + e] = part ? I : 1.0;\n                    double acc",
     "E[lid * 9 + e] = part ? -I : 1.0;\n                    double acc"),
    ("force_Yt_without_dagger", "orc_m5inv(p, (double *)Y, (double *)Yt, 1);",
     "orc_m5inv(p, (double *)Y, (double *)Yt, 0);"),
    ("force_W_hop_not_adjoint", "orc_hop(p, U, 0, (double *)Yt, (double *)t, 1);",
     "orc_hop(p, U, 0, (double *)Yt, (double *)t, 0);"),
    ("force_odd_row_fields_swapped", "acc += hop_overlap(p, E, Yt, Z, &sites[j], 1, tmp, buf);",
     "acc += hop_overlap(p, E, W, Z, &sites[j], 1, tmp, buf);"),
    ("dw_sites_mask_other_parity", "masked_copy(p, (const cplx *)ind, in_parity);",
     "masked_copy(p, (const cplx *)ind, in_parity < 0 ? in_parity : 1 - in_parity);"),
    ("dw_sites_adjoint_dropped", "dw_site(p, U, in, sites[k], tmp, dag, buf);",
     "dw_site(p, U, in, sites[k], tmp, 0, buf);"),
    ("sdep_adjoint_row_coefficient", "y[k] = c5_of(p, sm1) * t2[k]", "y[k] = c5_of(p, s) * t2[k]"),
    ("sdep_forward_row_coefficient", "o[k] += c5_of(p, s) * t2[k] - slice_buf[x * SITE_DOF + k];\n        } else {",
     "o[k] += c5_of(p, (s + 1) % Ls) * t2[k] - slice_buf[x * SITE_DOF + k];\n        } else {"),
    ("sdep_corner_coefficients_swapped",
     "km = -p->mf * Mm[Ls - 1];\n        kp = -p->mf * Mm[0];\n    } else {",
     "km = -p->mf * Mm[0];\n        kp = -p->mf * Mm[Ls - 1];\n    } else {"),
    ("sdep_adjoint_offdiagonal_index", "em[s] = s > 0 ? Mm[s - 1] : 0.0;", "em[s] = Mm[s];"),
    ("wall_force_pv_term_sign",
     "d[part] = -hopping_overlap(p, E, Z, chi, psi, at, 2, tmp, tmp0, buf) +",
     "d[part] = -hopping_overlap(p, E, Z, chi, psi, at, 2, tmp, tmp0, buf) -"),
    ("wall_force_pv_mass", "hopping_overlap(&pv, E, Z, chi, d1c", "hopping_overlap(p, E, Z, chi, d1c"),
    ("schur_right_inner_dagger", "orc_m5inv(p, (double *)xo, (double *)t1, 0);      /* I^-1        (odd)  */",
     "orc_m5inv(p, (double *)xo, (double *)t1, 1);      /* I^-1        (odd)  */"),
    ("adjoint_system_forward_block", "orc_hop(p, U, 1, (double *)t1, (double *)t2, dg);      /* odd <- even block",
     "orc_hop(p, U, 1, (double *)t1, (double *)t2, 0);      /* odd <- even block"),
    ("left_form_coefficient_row", "y[k] = c5_of(p, sm1) * W[sm1 * SITE_DOF + k]",
     "y[k] = c5_of(p, s) * W[sm1 * SITE_DOF + k]"),
    ("left_form_projector_swapped", "chiral_part(y, +1, fm1, o);\n            for",
     "chiral_part(y, -1, fm1, o);\n            for"),
    ("force_only_forward_site", "const int64_t sites[2] = {y, neighbour(p, y, mu, +1)};",
     "const int64_t sites[2] = {y, y};"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(orc, tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    hdr_dir = os.path.dirname(SRC)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-I", hdr_dir,
                    "-o", str(so), str(mut), "-lm"], check=True)
    caught = None
    with orc.using(str(so)):
        for pin in pins.ALL_PINS:
            try:
                pin(orc)
            except AssertionError:
                caught = pin.__name__
                break
    assert caught is not None, f"planted mistake {name} passed every pin"
