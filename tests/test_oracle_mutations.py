"""Planted mistakes in the oracle, on the CPU.

Each case copies oracle/oracle.c with one plausible mistake (a dropped term,
a flipped sign, a wrong coefficient, weight or index), builds that copy into
its own library and runs the pin that should notice it: every copy must fail
its pin, and the unmodified copy must pass all of them.  The pins compare
with closed forms, printed values and invariants, not with the oracle's own
formulas, so this shows that a mistake in each of these parts of the method
would not go unseen.  A copy counts as caught only when its pin fails an
assertion (a copy that does not build, or a test that errors, does not
count)."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

SP = "tests/test_oracle_spatial.py::"
RU = "tests/test_oracle_rules.py::"
IM = "tests/test_oracle_imex.py::"
PT = "tests/test_oracle_point.py::"
GL = "tests/test_oracle_glm.py::"
UI = "tests/test_oracle_uct_ideal.py::"
DY = "tests/test_oracle_dynamo.py::"

# (what is planted, the text it replaces, the replacement, the pin)
MUTATIONS = [
    ("HLL dissipation with the wrong sign (Sec 2.5)",
     "F[v] = (cp * fL[v] + cm * fR[v] - cp * cm * (qR[v] - qL[v])) / (cp + cm);",
     "F[v] = (cp * fL[v] + cm * fR[v] + cp * cm * (qR[v] - qL[v])) / (cp + cm);",
     DY + "test_printed_growth_k1"),
    ("upwind EMF jump of q_B^b reversed (Sec 3.2 (vii))",
     "cap * cam / (cap + cam) * (qbR - qbL) - cbp * cbm / (cbp + cbm) * (qaR - qaL);",
     "cap * cam / (cap + cam) * (qbL - qbR) - cbp * cbm / (cbp + cbm) * (qaR - qaL);",
     DY + "test_printed_growth_k1"),
    ("edge lapse replaced by 1 (Sec 3.2 (v))",
     "double ae = asum / na;", "double ae = 1.0 + 0.0 * asum / na;",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("non-stiff current rho_e v with the wrong sign (Sec 2.1)",
     "for (int a = 0; a < 3; a++) L[5 + a] += -al * m.sqrtg * rhoe * v[a];\n                for (int vv",
     "for (int a = 0; a < 3; a++) L[5 + a] += al * m.sqrtg * rhoe * v[a];\n                for (int vv",
     SP + "test_gauss_charge_current_closed_form"),
    ("metric-derivative source of S_i dropped (Sec 2.1)",
     "sg += 0.5 * al * Sjk[jj][kk] * dg;", "sg += 0.0 * al * Sjk[jj][kk] * dg;",
     SP + "test_tov_hydrostatic_residual_converges"),
    ("energy source s_tau dropped (Sec 2.1)",
     "L[4] += m.sqrtg * st;", "L[4] += 0.0 * st;",
     SP + "test_killing_energy_in_static_lapse"),
    ("IMEX-SSP3(4,3,3) explicit coefficient a~_31 mistyped (Sec 2.3)",
     "At[3 * 4 + 1] = 0.25;", "At[3 * 4 + 1] = 0.26;",
     IM + "test_ssp3_order_conditions"),
    ("PPM interface weight 1/6 for 1/12",
     "double v = 7.0 / 12.0 * (a0 + a1) - 1.0 / 12.0 * (am1 + a2);",
     "double v = 7.0 / 12.0 * (a0 + a1) - 1.0 / 6.0 * (am1 + a2);",
     IM + "test_recon_exact_on_linear_data"),
    ("PPM steepening threshold d^2/3 for d^2/6",
     "if (d * mm > d * d / 6.0) *aL = 3.0 * a - 2.0 * *aR;",
     "if (d * mm > d * d / 3.0) *aL = 3.0 * a - 2.0 * *aR;",
     IM + "test_recon_reflection_symmetry_and_bounds"),
    ("eq. im_E coefficient A_1 without its factor W (Sec 2.4)",
     "c->A[1] = et / opW + x2 * et * W / (Wpe * opW);", "c->A[1] = et / opW + x2 * et / (Wpe * opW);",
     PT + "test_im_E_coefficients_match_direct_solve"),
    ("eq. im_E coefficient A_2 with the wrong sign (Sec 2.4)",
     "c->A[2] = -xi * et / Wpe;", "c->A[2] = xi * et / Wpe;",
     PT + "test_im_E_coefficients_match_direct_solve"),
    ("GLM damping kappa_E of Psi dropped (Sec 3.1)",
     "L[11] += m.sqrtg * (al * rhoe - al * G->kappa_E * Psi + Eda);", "L[11] += m.sqrtg * (al * rhoe + Eda);",
     GL + "test_uniform_psi_phi_decay_at_the_explicit_rate"),
    ("GLM damping kappa_B of Phi with the wrong sign (Sec 3.1)",
     "L[12] += m.sqrtg * (-al * G->kappa_B * Phi + Bda);", "L[12] += m.sqrtg * (al * G->kappa_B * Phi + Bda);",
     GL + "test_glm_wave_closed_form"),
    ("ideal-MHD EMF: face velocities weighted by the wrong sides (App. A)",
     "return (cm * vR + cp * vL) / (cm + cp);", "return (cm * vL + cp * vR) / (cm + cp) + 1e-3 * (vR - vL);",
     UI + "test_ideal_uct_blast_wave_mirror_symmetry"),
    ("ideal-MHD EMF: b-direction term with the wrong sign (App. A)",
     "return -t1 + t2;", "return -t1 - t2;",
     UI + "test_linear_field_face_update_exact"),
    ("E of a cell at rest with the wrong relaxation factor (R23b)",
     "for (int i = 0; i < 3; i++) E[i] = (Es[i] + xi * r * B[i]) / (1.0 + r);",
     "for (int i = 0; i < 3; i++) E[i] = (Es[i] + xi * r * B[i]) / (1.0 + 2.0 * r);",
     RU + "test_fallback_state_field_and_count"),
    ("atmosphere pressure set to the atmosphere density (R18)",
     "prim[4] = G->p_atm;", "prim[4] = G->rho_atm;",
     RU + "test_fallback_state_field_and_count"),
    ("resistivity not clamped at eta_min (eq. sigma_D)",
     "return e < G->eta_min ? G->eta_min : e;", "return e;",
     RU + "test_eta_of_D_from_relaxation"),
    ("outflow ghost copied from the second interior cell (R17)",
     "s[d] = (bc == BC_PERIODIC) ? m + n : g;\n                        } else {",
     "s[d] = (bc == BC_PERIODIC) ? m + n : g + 1;\n                        } else {",
     RU + "test_ghost_fill_rules"),
    ("CFL rate not summed over directions (R16)",
     "s += al * sqrt(1.0 / pow4(ps)) / q.dx[d];", "s = al * sqrt(1.0 / pow4(ps)) / q.dx[d];",
     RU + "test_cfl_dt_flat_closed_form"),
    ("minmod picks the larger slope",
     "return (fabs(a) < fabs(b)) ? a : b;", "return (fabs(a) > fabs(b)) ? a : b;",
     IM + "test_recon_reflection_symmetry_and_bounds"),
    ("minmod right state extrapolated to the wrong side",
     "*R = w[3] - 0.5 * minmod2(w[3] - w[2], w[4] - w[3]);", "*R = w[3] + 0.5 * minmod2(w[3] - w[2], w[4] - w[3]);",
     IM + "test_recon_exact_on_linear_data"),
    ("MC centred slope without its 1/2",
     "return minmod3(0.5 * (r - l), 2.0 * (c - l), 2.0 * (r - c));",
     "return minmod3((r - l), 2.0 * (c - l), 2.0 * (r - c));",
     DY + "test_printed_growth_k1"),
    ("MC one-sided slope factor 1 for 2",
     "return minmod3(0.5 * (r - l), 2.0 * (c - l), 2.0 * (r - c));",
     "return minmod3(0.5 * (r - l), 1.0 * (c - l), 2.0 * (r - c));",
     DY + "test_closed_form_growth_k2"),
    ("PPM interface value not clipped between its neighbours",
     "    if (v < lo) v = lo;\n    if (v > hi) v = hi;\n    return v;", "    (void)lo;\n    (void)hi;\n    return v;",
     IM + "test_recon_reflection_symmetry_and_bounds"),
    ("CT face update with the wrong sign (eq. ct)",
     "Lf[d][id] = -s;", "Lf[d][id] = s;",
     DY + "test_printed_growth_k1"),
    ("CT face update with transposed Levi-Civita indices (eq. ct)",
     "double e = levi(d, m, kk);", "double e = levi(m, d, kk);",
     DY + "test_printed_growth_k1"),
    ("periodic ghost image one cell off (R17)",
     "s[d] = (bc == BC_PERIODIC) ? m + n : g;\n                        } else {",
     "s[d] = (bc == BC_PERIODIC) ? m + n - 1 : g;\n                        } else {",
     DY + "test_printed_growth_k1"),
    ("stage faces built with the implicit weights (Sec 2.3)",
     "for (int j = 0; j < i; j++) acc += dt * At[i * 4 + j] * Lf[j][d][id];",
     "for (int j = 0; j < i; j++) acc += dt * A[i * 4 + j] * Lf[j][d][id];",
     DY + "test_printed_growth_k1"),
    ("final face update missing the last stage (Sec 2.3)",
     "for (int j = 0; j < s; j++) acc += dt * wt[j] * Lf[j][d][id];",
     "for (int j = 0; j < s - 1; j++) acc += dt * wt[j] * Lf[j][d][id];",
     DY + "test_printed_growth_k1"),
    ("final weight of the last SSP3 stage dropped (Sec 2.3)",
     "for (int i = 0; i < 4; i++) w[i] = wt[i];", "for (int i = 0; i < 3; i++) w[i] = wt[i];",
     IM + "test_ssp3_order_conditions"),
    ("IMEX-SSP2(2,2,2) gamma 1 - 1/sqrt(3) (Table imex_ssp2)",
     "double g = 1.0 - 1.0 / sqrt(2.0);", "double g = 1.0 - 1.0 / sqrt(3.0);",
     IM + "test_ssp2_tableau_is_the_printed_one"),
    ("implicit stage without the lapse in eta~ (Sec 2.4)",
     "double etat = eta / (al * aii * dt);", "double etat = eta / (aii * dt);",
     IM + "test_stiff_relaxation_amplification"),
    ("frozen-matter E without the lapse in eta~ (Sec 5.7)",
     "or_implicit_E(ps, eta / (al * aii * dt), G->xi, ut, Es, B, E);",
     "or_implicit_E(ps, eta / (aii * dt), G->xi, ut, Es, B, E);",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("Gauss-law charge from psi^4 E instead of q_E = psi^6 E (Sec 2.1)",
     "double qEp = pow6(P_at(&c, ip)) * E[d][ip], qEm = pow6(P_at(&c, im)) * E[d][im];\n                    divqE",
     "double qEp = pow4(P_at(&c, ip)) * E[d][ip], qEm = pow4(P_at(&c, im)) * E[d][im];\n                    divqE",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("eq. im_E dynamo coefficient A_3 without (1 + W) (Sec 2.4)",
     "c->A[3] = xi * opW / Wpe;", "c->A[3] = xi / Wpe;",
     DY + "test_printed_growth_k1"),
    ("eq. im_E dynamo coefficient A_4 without xi^2 (Sec 2.4)",
     "c->A[4] = xi * (1.0 - et * et + x2) / (Wpe * opW);", "c->A[4] = xi * (1.0 - et * et) / (Wpe * opW);",
     PT + "test_im_E_coefficients_match_direct_solve"),
    ("recovery: internal energy with the wrong pressure sign (Sec 2.6)",
     "double rhoeps = (tauf + D * (1.0 - W) + p * (1.0 - W * W)) / (W * W);",
     "double rhoeps = (tauf + D * (1.0 - W) - p * (1.0 - W * W)) / (W * W);",
     PT + "test_prim_cons_round_trip"),
    ("GLM source E^i d_i alpha of Psi dropped (Sec 3.1)",
     "L[11] += m.sqrtg * (al * rhoe - al * G->kappa_E * Psi + Eda);",
     "L[11] += m.sqrtg * (al * rhoe - al * G->kappa_E * Psi);",
     GL + "test_lapse_gradient_sources_balance_the_fluxes"),
    ("GLM source B^i d_i alpha of Phi dropped (Sec 3.1)",
     "L[12] += m.sqrtg * (-al * G->kappa_B * Phi + Bda);", "L[12] += m.sqrtg * (-al * G->kappa_B * Phi);",
     GL + "test_lapse_gradient_sources_balance_the_fluxes"),
    ("GLM charge source alpha rho_e of Psi dropped (Sec 3.1)",
     "L[11] += m.sqrtg * (al * rhoe - al * G->kappa_E * Psi + Eda);",
     "L[11] += m.sqrtg * (-al * G->kappa_E * Psi + Eda);",
     GL + "test_charge_source_balances_the_divergence_of_E"),
    ("GLM gradient of Psi in the E equation dropped (Sec 3.1)",
     "L[5 + a] += -al * m.sqrtg * gPsi;", "L[5 + a] += 0.0 * gPsi;",
     GL + "test_psi_drives_E_and_decays"),
    ("GLM gradient of Phi in the B equation dropped (Sec 3.1)",
     "L[8 + a] += -al * m.sqrtg * gPhi;", "L[8 + a] += 0.0 * gPhi;",
     GL + "test_glm_wave_closed_form"),
    ("GLM flux of q_Psi without the lapse (Sec 3.1)",
     "ff[11] = al * p6 * E[d];", "ff[11] = p6 * E[d];",
     GL + "test_lapse_gradient_sources_balance_the_fluxes"),
    ("GLM flux of q_Phi without the lapse (Sec 3.1)",
     "ff[12] = al * p6 * B[d];", "ff[12] = p6 * B[d];",
     GL + "test_lapse_gradient_sources_balance_the_fluxes"),
    ("momentum flux with twice the electromagnetic pressure (Sec 2.1)",
     "double Sij = (p + 0.5 * (E2 + B2)) * (i == j ? 1.0 : 0.0)", "double Sij = (p + (E2 + B2)) * (i == j ? 1.0 : 0.0)",
     SP + "test_charged_vortex_matches_paper_table"),
    ("energy flux without -v^i D (Sec 2.1)",
     "f[4] = m.sqrtg * alpha * (Su[i] - v[i] * D);", "f[4] = m.sqrtg * alpha * Su[i];",
     SP + "test_star_div_b_round_off"),
    ("flux of q_E with the wrong sign (Sec 2.1)",
     "f[5 + j] = -m.sqrtg * s;", "f[5 + j] = m.sqrtg * s;",
     DY + "test_printed_growth_k1"),
    ("flux of q_D with rho for D (Sec 2.1)",
     "f[0] = m.sqrtg * D * vhat;", "f[0] = m.sqrtg * rho * vhat;",
     SP + "test_density_wave_second_order"),
    ("Gauss-law charge divergence without its 1/2 (Sec 2.1)",
     "divqE += (qEp - qEm) / (2.0 * q->dx[d]);", "divqE += (qEp - qEm) / (q->dx[d]);",
     SP + "test_gauss_charge_current_closed_form"),
    ("charge density without 1/psi^6 (Sec 2.1)",
     "double rhoe = divqE / m.sqrtg;\n                for (int a = 0; a < 3; a++) L[5 + a]",
     "double rhoe = divqE;\n                for (int a = 0; a < 3; a++) L[5 + a]",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("W-derivative of the dynamo coefficient A_2 with the wrong sign (Sec 2.4)",
     "c->Ad[2] = xi * et / (Wpe * Wpe);", "c->Ad[2] = -xi * et / (Wpe * Wpe);",
     PT + "test_jacobian_matches_finite_differences"),
    ("tau without the electric energy (Sec 2.1)",
     "double tau = rho * h * W * W - p + 0.5 * (E2 + B2) - D;", "double tau = rho * h * W * W - p + 0.5 * (B2) - D;",
     PT + "test_prim_cons_round_trip"),
    ("momentum density without E x B (Sec 2.1)",
     "for (int j = 0; j < 3; j++) q[1 + j] = m.sqrtg * (rho * h * W * W * vl[j] + ExB[j]);",
     "for (int j = 0; j < 3; j++) q[1 + j] = m.sqrtg * (rho * h * W * W * vl[j]);",
     PT + "test_prim_cons_round_trip"),
    ("q_E without sqrt(gamma) (Sec 2.1)",
     "for (int j = 0; j < 3; j++) q[5 + j] = m.sqrtg * E[j];\n}", "for (int j = 0; j < 3; j++) q[5 + j] = E[j];\n}",
     RU + "test_fallback_state_field_and_count"),
    ("metric derivative d gamma = 2 psi^3 d psi for 4 psi^3 d psi (Sec 2.1)",
     "double dg = (jj == kk) ? 4.0 * ps * ps * ps * dps[a] : 0.0;",
     "double dg = (jj == kk) ? 2.0 * ps * ps * ps * dps[a] : 0.0;",
     SP + "test_tov_hydrostatic_residual_converges"),
    ("lapse-gradient force -(tau + D) d alpha dropped (Sec 2.1)",
     "L[1 + a] += m.sqrtg * (-tauD * dal[a] + sg);", "L[1 + a] += m.sqrtg * (sg);",
     SP + "test_tov_hydrostatic_residual_converges"),
    ("dynamo term of the at-rest field dropped (Sec 2.4)",
     "for (int i = 0; i < 3; i++) E[i] = (Es[i] + xi * r * B[i]) / (1.0 + r);",
     "for (int i = 0; i < 3; i++) E[i] = (Es[i]) / (1.0 + r);",
     RU + "test_fallback_field_with_the_dynamo_term"),
    ("GLM HLL speed without the lapse (Sec 2.5)",
     "double sp = al * sqrt(1.0 / pow4(ps));\n    for (int v = 0; v < GLM_NV; v++)",
     "double sp = sqrt(1.0 / pow4(ps));\n    for (int v = 0; v < GLM_NV; v++)",
     GL + "test_glm_constant_metric_is_a_rescaled_flat_run"),
    ("face conformal factor taken from one cell (Sec 2.5)",
     "    *al = 0.5 * (A_at(c, i0) + A_at(c, i1));\n    *ps = 0.5 * (P_at(c, i0) + P_at(c, i1));",
     "    *al = 0.5 * (A_at(c, i0) + A_at(c, i1));\n    *ps = P_at(c, i1);",
     SP + "test_uniform_pressure_in_a_conformal_factor_is_an_equilibrium"),
    ("face lapse taken from one cell (Sec 2.5)",
     "    *al = 0.5 * (A_at(c, i0) + A_at(c, i1));\n    *ps = 0.5 * (P_at(c, i0) + P_at(c, i1));",
     "    *al = A_at(c, i1);\n    *ps = 0.5 * (P_at(c, i0) + P_at(c, i1));",
     SP + "test_killing_energy_in_static_lapse"),
    ("face speed alpha / psi^4 for alpha / psi^2 (Sec 2.5)",
     "return al / (ps * ps);", "return al / (ps * ps * ps * ps);",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("E at the a-faces without psi^4 (Sec 3.2 (ii))",
     "    *L = l * p4;\n    *R = r * p4;", "    *L = l;\n    *R = r;",
     SP + "test_constant_metric_is_a_rescaled_flat_run"),
    ("cell-centred B without 1/psi^6",
     "B[d] = 0.5 * (face[d][id] + face[d][IXv(q, cp)]) / p6;", "B[d] = 0.5 * (face[d][id] + face[d][IXv(q, cp)]);",
     RU + "test_fallback_field_with_the_dynamo_term"),
    ("cell-centred B from one face",
     "B[d] = 0.5 * (face[d][id] + face[d][IXv(q, cp)]) / p6;", "B[d] = face[d][id] / p6;",
     RU + "test_final_recovery_rewrites_conserved_variables"),
    ("stiff term R without psi^6 (Sec 2.3)",
     "R[i][a][id] = (p6 * E[a] - qs[5 + a]) / (aii * dt);", "R[i][a][id] = (E[a] - qs[5 + a]) / (aii * dt);",
     IM + "test_stiff_relaxation_amplification"),
    ("stage cells with the implicit weights on L (Sec 2.3)",
     "acc += dt * At[i * 4 + j] * Lc[j][v][id];\n                            if (v >= 5)",
     "acc += dt * A[i * 4 + j] * Lc[j][v][id];\n                            if (v >= 5)",
     DY + "test_closed_form_growth_k2"),
    ("stage cells with the explicit weights on R (Sec 2.3)",
     "if (v >= 5) acc += dt * A[i * 4 + j] * R[j][v - 5][id];",
     "if (v >= 5) acc += dt * At[i * 4 + j] * R[j][v - 5][id];",
     DY + "test_closed_form_growth_k2"),
    ("edge speed along a: the slower of the two a-faces (Sec 3.2 (vi))",
     "*ca = fmax(face_speed(c, a, c1), face_speed(c, a, c2));",
     "*ca = fmin(face_speed(c, a, c1), face_speed(c, a, c2));",
     SP + "test_edge_speed_is_that_of_the_faster_face"),
    ("edge speed along b: the slower of the two b-faces (Sec 3.2 (vi))",
     "*cb = fmax(face_speed(c, b, c3), face_speed(c, b, c4));",
     "*cb = fmin(face_speed(c, b, c3), face_speed(c, b, c4));",
     SP + "test_edge_speed_is_that_of_the_faster_face"),
    ("L1 norm of div B summed, not averaged (eq. divb_0)",
     "    out[0] = s1 / cnt;\n    out[1] = sqrt(s2 / cnt);\n    out[2] = mx;\n}\n\n\n",
     "    out[0] = s1;\n    out[1] = sqrt(s2 / cnt);\n    out[2] = mx;\n}\n\n\n",
     SP + "test_div_b_norms_of_a_known_divergence"),
    ("face divergence with a sum for a difference (eq. divb_0)",
     "dv += (face[d][IXv(&q, cp)] - face[d][id]) / q.dx[d];", "dv += (face[d][IXv(&q, cp)] + face[d][id]) / q.dx[d];",
     SP + "test_div_b_norms_of_a_known_divergence"),
    ("cell-centred divergence without the 1/2 of the central difference",
     "dv += (tmp[d][IXv(&q, cp)] - tmp[d][IXv(&q, cm)]) / (2.0 * q.dx[d]);",
     "dv += (tmp[d][IXv(&q, cp)] - tmp[d][IXv(&q, cm)]) / (q.dx[d]);",
     GL + "test_div_b_norms_of_cell_centred_field"),
    ("recovery: E x B not removed from S (Sec 2.6)",
     "for (int j = 0; j < 3; j++) Sf[j] = S[j] - ExB[j];", "for (int j = 0; j < 3; j++) Sf[j] = S[j];",
     PT + "test_prim_cons_round_trip"),
    ("recovery: electromagnetic energy not removed from tau (Sec 2.6)",
     "double tauf = tau - UEM;", "double tauf = tau;",
     IM + "test_stiff_relaxation_amplification"),
    ("recovery: u~ without its factor W (Sec 2.6)",
     "for (int i = 0; i < 3; i++) prim[1 + i] = W * Sfu[i] / Z;", "for (int i = 0; i < 3; i++) prim[1 + i] = Sfu[i] / Z;",
     PT + "test_prim_cons_round_trip"),
    ("recovery: rho = D (Sec 2.6)",
     "prim[0] = D / W;", "prim[0] = D;",
     PT + "test_prim_cons_round_trip"),
    ("CFL speed without 1/psi^2 (Sec 2.5)",
     "if (q.act[d]) s += al * sqrt(1.0 / pow4(ps)) / q.dx[d];", "if (q.act[d]) s += al / q.dx[d];",
     RU + "test_cfl_dt_constant_metric_is_rescaled_flat_step"),
    ("CFL speed without the lapse (Sec 2.5)",
     "if (q.act[d]) s += al * sqrt(1.0 / pow4(ps)) / q.dx[d];", "if (q.act[d]) s += sqrt(1.0 / pow4(ps)) / q.dx[d];",
     RU + "test_cfl_dt_constant_metric_is_rescaled_flat_step"),
    ("reconstruction stencil shifted by one cell",
     "        cc[d] += m - 3;\n        if (kind != RC_PPM && (m == 0 || m == 5)) { w[m] = 0.0; continue; }",
     "        cc[d] += m - 2;\n        if (kind != RC_PPM && (m == 0 || m == 5)) { w[m] = 0.0; continue; }",
     DY + "test_printed_growth_k1"),
]


def _run(workdir, text, pins):
    os.makedirs(workdir, exist_ok=True)
    src = os.path.join(workdir, "oracle.c")
    with open(src, "w") as f:
        f.write(text)
    # build the copy first (the same command as oracle.build): a copy that
    # does not compile is reported as such, never as caught
    b = subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o",
                        os.path.join(workdir, "liboracle.so"), src, "-lm"], capture_output=True, text=True)
    if b.returncode != 0:
        return -1, "build failed:\n" + b.stderr[-2000:]
    env = dict(os.environ, GR_ORACLE_SRC=src, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-3000:]


def test_planted_mistakes_fail_their_pins(tmp_path):
    base = open(SRC).read()
    for what, old, new, pin in MUTATIONS:
        assert base.count(old) >= 1, "no longer in the oracle: %s" % what
    pins = sorted({m[3] for m in MUTATIONS})
    jobs = [("unmodified", base, pins)] + [(m[0], base.replace(m[1], m[2], 1), [m[3]]) for m in MUTATIONS]
    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(_run, str(tmp_path / ("m%d" % i)), text, p) for i, (_, text, p) in enumerate(jobs)]
        res = [f.result() for f in futs]
    rc0, out0 = res[0]
    assert rc0 == 0, "the unmodified oracle fails its pins:\n" + out0
    def caught(rc, out):
        tail = out.strip().splitlines()[-1] if out.strip() else ""
        return rc == 1 and " failed" in tail and " error" not in tail

    missed = [jobs[i][0] for i in range(1, len(jobs)) if not caught(*res[i])]
    for i in range(1, len(jobs)):
        print("%-8s %s" % ("caught" if caught(*res[i]) else "MISSED", jobs[i][0]))
    assert not missed, missed
