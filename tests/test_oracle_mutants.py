"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it, and checks that at least one pin of test_oracle_pins,
test_oracle_force or test_oracle_tables fails
against the broken build.  Only memory-safe mutations are planted."""
import os

import numpy as np
import pytest

import oracle
from tests import test_oracle_force as force_pins
from tests import test_oracle_pins as pins
from tests import test_oracle_tables as table_pins

MUTANTS = {
    "eta_all_one": ("return (s & 1) ? -1.0 : 1.0;", "return 1.0;"),
    "eta_wrong_range": ("for (int nu = 0; nu < mu; ++nu) s += x[nu];",
                        "for (int nu = 0; nu <= mu; ++nu) s += x[nu];"),
    "drop_backward_hop": ("add_mul_dag(acc, -e * bc_sign(g, mu, z), link_at(g, U, mu, lz), vz);",
                          ";"),
    "backward_sign": ("add_mul_dag(acc, -e * bc_sign(g, mu, z)", "add_mul_dag(acc, e * bc_sign(g, mu, z)"),
    "backward_no_conj": ("s += conj(U[b * 3 + a]) * v[b];", "s += U[b * 3 + a] * v[b];"),
    "forward_transposed": ("s += U[a * 3 + b] * v[b];", "s += U[b * 3 + a] * v[b];"),
    "backward_link_at_x": ("link_at(g, U, mu, lz), vz)", "link_at(g, U, mu, coord_to_lex(g, x)), vz)"),
    "bc_sign_wrong_site": ("-e * bc_sign(g, mu, z)", "-e * bc_sign(g, mu, x)"),
    "periodic_time": ("(g->antiperiodic_t && mu == 3", "(0 && mu == 3"),
    "no_half": ("out[a] = 0.5 * acc[a];", "out[a] = acc[a];"),
    "mass_not_squared": ("double c = mass * mass + shift;", "double c = mass + shift;"),
    "zeta_shift_sign": ("(1.0 + s * alpha)", "(1.0 - s * alpha)"),
    "zeta_history_swapped": ("alpha * beta_prev * (zeta_prev[i] - zeta[i])",
                             "alpha * beta_prev * (zeta[i] - zeta_prev[i])"),
    "beta_i_unsquared": ("bi = beta * ratio * ratio", "bi = beta * ratio"),
    "alpha_i_inverted": ("double ai = alpha * ratio,", "double ai = alpha / ratio,"),
    "x_update_uses_r": ("xi[j] += ai * pi[j];", "xi[j] += ai * r[j];"),
    "force_odd_end_sign": ("(odd ? -0.5 : 0.5)", "(odd ? 0.5 : 0.5)"),
    "force_outer_swapped": ("W[a * 3 + b] += k * left[a] * conj(right[b]);",
                            "W[a * 3 + b] += k * right[a] * conj(left[b]);"),
    "force_no_eta": ("const double es = eta(mu, c) * bc_sign(&g, mu, c);",
                     "const double es = bc_sign(&g, mu, c);"),
    "force_w_times_u": ("s += u[a * 3 + e] * W[e * 3 + b];", "s += W[a * 3 + e] * u[e * 3 + b];"),
    "force_y_unsigned": ("y[i * n + k] = -y[i * n + k];", "y[i * n + k] = y[i * n + k];"),
    "force_trace_kept": ("(a == b ? tr / 6.0 : 0)", "(a == b ? 0.0 * tr : 0)"),
    "tables_bwd_sign_at_x": ("sign[(p * 8 + 4 + mu) * g.Vh + i] = (int32_t)(eta(mu, x) * bc_sign(&g, mu, z));",
                             "sign[(p * 8 + 4 + mu) * g.Vh + i] = (int32_t)(eta(mu, x) * bc_sign(&g, mu, x));"),
    "tables_fwd_slot_gets_bwd": ("nbr[(p * 8 + mu) * g.Vh + i] = (int32_t)(coord_to_lex(&g, y) >> 1);",
                                 "nbr[(p * 8 + mu) * g.Vh + i] = (int32_t)(coord_to_lex(&g, z) >> 1);"),
    "tables_coord_reversed": ("coord[(p * g.Vh + i) * 4 + mu] = x[mu];",
                              "coord[(p * g.Vh + i) * 4 + mu] = x[3 - mu];"),
    "tables_parity_from_x0": ("int p = site_parity(x);", "int p = x[0] & 1;"),
}


def _pin_cases(o):
    yield lambda: pins.test_free_field_plane_wave_eigen(o, (4, 4, 4, 4), True)
    yield lambda: pins.test_free_field_plane_wave_eigen(o, (6, 4, 2, 8), True)
    yield lambda: pins.test_anti_hermitian(o, (4, 4, 4, 4))
    yield lambda: pins.test_parity_mapping(o, (4, 4, 4, 4), 1)
    yield lambda: pins.test_gauge_covariance(o, (6, 4, 2, 8))
    yield lambda: pins.test_translation_by_two(o, (6, 4, 2, 8), 0)
    yield lambda: pins.test_multishift_free_field_closed_form(o, (4, 4, 4, 4))
    yield lambda: pins.test_multishift_dense_solve(o, (2, 2, 2, 2), 1)
    yield lambda: pins.test_multishift_iterated_equals_true_residual_early(o)
    yield lambda: force_pins.test_force_is_the_action_derivative(o, (4, 2, 2, 4), True)
    yield lambda: force_pins.test_force_is_in_the_algebra_and_linear_in_alpha(o)
    yield lambda: table_pins.test_tables_match_numpy_geometry(o, (6, 4, 2, 8), True)


def _failures(o):
    n = 0
    for case in _pin_cases(o):
        try:
            case()
        except (AssertionError, ValueError, FloatingPointError, np.linalg.LinAlgError):
            n += 1
    return n


def test_pins_pass_on_unmodified_source(tmp_path):
    srcs = [os.path.join(oracle._HERE, f) for f in oracle.SOURCES
            if os.path.exists(os.path.join(oracle._HERE, f))]
    o = oracle.load(oracle.compile_sources(srcs, str(tmp_path / "liborc_ref.so")))
    assert _failures(o) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(oracle._HERE, "orc.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    path = tmp_path / "orc_mut.c"
    path.write_text(src.replace(old, new))
    o = oracle.load(oracle.compile_sources([str(path)], str(tmp_path / f"liborc_{name}.so")))
    assert _failures(o) >= 1, f"no pin caught mutant {name}"
