"""Planted mistakes in copies of the oracle, each paired with the pins that
must catch it.  Used by ``test_oracle_mutations.py`` (a CPU-only test): every
mutant is compiled from a copy of ``oracle/lbm_oracle.c`` with one textual
change and the named pins are run against it; each must fail.

Every entry: (name, original text, replacement, occurrences replaced, pytest -k
expression selecting the pins in test_oracle_pins.py that catch it).
"""

MUTATIONS = [
    # Spalart-Allmaras right-hand side (Sec. 2.2, eq. 11-14)
    ("sa_fw_exponent", "pow((1.0 + cw36) / (g6 + cw36), 1.0 / 6.0)",
     "pow((1.0 + cw36) / (g6 + cw36), 1.0 / 3.0)", 1,
     "negative_s_tilde or wall_distance_follows"),
    ("sa_fv2_dropped", "double St = S + nt0 / (k * k * d * d) * fv2;",
     "double St = S + nt0 / (k * k * d * d);", 1, "constant_stress_layer"),
    ("sa_r_zero_when_s_tilde_negative", "P = 0.0;\n        r = p->rlim;",
     "P = 0.0;\n        r = 0.0;", 1, "negative_s_tilde or wall_distance_follows"),
    ("sa_g_power_five", "gg = r + p->cw2 * (pow(r, 6.0) - r)", "gg = r + p->cw2 * (pow(r, 5.0) - r)", 1,
     "destruction_slope"),
    ("sa_cw2_dropped", "gg = r + p->cw2 * (pow(r, 6.0) - r)", "gg = r", 1, "destruction_slope"),
    ("sa_fv1_square", "double fv1 = chi3 / (chi3 + cv13);", "double fv1 = chi * chi / (chi * chi + cv13);",
     1, "constant_stress_layer"),
    ("sa_cw1_sign", "double cw1 = p->cb1 / (k * k) + (1.0 + p->cb2) / p->sigma;",
     "double cw1 = p->cb1 / (k * k) + (1.0 - p->cb2) / p->sigma;", 1, "log_layer or constant_stress"),
    ("sa_cb2_dropped", "return -conv + P - Dst + (diff + p->cb2 * grad2) / p->sigma;",
     "return -conv + P - Dst + diff / p->sigma;", 1, "log_layer or diffusion_second_order"),
    ("sa_diffusion_face_upwind", "diff += (nu + 0.5 * (ntp[a] + nt0)) * (ntp[a] - nt0)",
     "diff += (nu + ntp[a]) * (ntp[a] - nt0)", 1, "diffusion_second_order"),
    ("sa_upwind_direction", "if (ua > 0.0)\n            conv += ua * (nt0 - ntm[a]);",
     "if (ua < 0.0)\n            conv += ua * (nt0 - ntm[a]);", 1, "sa_rhs_terms"),
    ("sa_production_missing_nt", "P = p->cb1 * St * nt0;", "P = p->cb1 * St;", 1, "log_layer"),
    ("sa_nut_exponent", "return nt * chi3 / (chi3 + cv13);", "return nt * chi * chi / (chi * chi + cv13);", 1,
     "sa_rhs_terms"),
    # collision and forcing (Sec. 2.1, eq. 2, 5, 7)
    ("guo_prefactor_sign", "src *= (1.0 - 0.5 * omega) * w[i];", "src *= (1.0 + 0.5 * omega) * w[i];", 1,
     "poiseuille_closed_form or collision_conserves"),
    ("half_force_shift_dropped", "for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * force[a]) / rho;\n    orc_feq",
     "for (int a = 0; a < 3; ++a) u[a] = m[a] / rho;\n    orc_feq", 1, "collision_conserves"),
    ("cm_trace_relaxed", "ks[j] = rho * CS2 + (1.0 - omega) * (k[j] - tr / D);",
     "ks[j] = rho * CS2 + (1.0 - omega) * k[j];", 1, "cm_"),
    ("cm_third_order_forcing", "ks[j] = 0.5 * CS2 * force[b];", "ks[j] = 0.0;", 1, "cm_forcing"),
    ("cm_fourth_order_equilibrium", "ks[j] = rho * CS2 * CS2;", "ks[j] = rho * CS2;", 1, "cm_"),
    # wall laws (eq. 15-16, Reichardt) and the friction-velocity solve (Sec. 3.1)
    ("reichardt_constant", "double C = B - log(kappa) / kappa;\n    return log(1.0 + kappa * yp)",
     "double C = B;\n    return log(1.0 + kappa * yp)", 1, "reichardt"),
    ("sa_law_bbar_printed", "static const double SA_BBAR = 5.0333908790505579;",
     "static const double SA_BBAR = 5.033908790505579;", 1, "eq16"),
    ("sa_law_plain_arctan", "- SA_C3 * atan2(SA_B1, yp + SA_A1) -\n               SA_C4 * atan2(SA_B2, yp + SA_A2)",
     "- SA_C3 * atan(SA_B1 / (yp + SA_A1)) -\n               SA_C4 * atan(SA_B2 / (yp + SA_A2))", 1, "eq16"),
    # bounce-back family (Sec. 3.2, eq. 31, 35-37)
    ("bounce_back_moving_wall_sign", "val = o->fpost[io * N + cell] - 2.0 * o->w[io] * rho_w * cu / CS2;",
     "val = o->fpost[io * N + cell] + 2.0 * o->w[io] * rho_w * cu / CS2;", 1, "couette_exact"),
    ("slip_law_nut_dropped", "double s = ut_ * ut_ * yB / (p->nu * (1.0 + p->kappa * yBp));",
     "double s = ut_ * ut_ * yB / p->nu;", 1, "slip_bounce_back_laminar"),
    ("bouzidi_weight", "fr = 2.0 * q * fkB + (1.0 - 2.0 * q) * fkF - corr;",
     "fr = 2.0 * q * fkB + (1.0 - q) * fkF - corr;", 1, "ibb_couette or ibb_poiseuille"),
    ("bouzidi_moving_wall_term", "fr = fkB / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * frB - corr / (2.0 * q);",
     "fr = fkB / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * frB - corr;", 1, "ibb_couette"),
    ("yu_back_interpolation", "fr = frW + q / (1.0 + q) * (frB - frW);", "fr = frW + q / (2.0 + q) * (frB - frW);",
     1, "ibb_couette or ibb_poiseuille"),
    ("yu_wall_point", "const double frW = q * fkB + (1.0 - q) * fkF - corr;",
     "const double frW = 0.5 * fkB + 0.5 * fkF - corr;", 1, "ibb_couette or ibb_poiseuille"),
    ("wall_distance_ignores_q", "double yc = y + dw;", "double yc = y + 0.5;", 1, "wall_distance_follows"),
    ("reference_node_ignores_q", "yF = 1.0 + p->wall_dist; /* Sec. 3.1: B and F */",
     "yF = 1.5; /* Sec. 3.1: B and F */", 1, "reference_node_follows"),
    # regularized reconstruction (Sec. 3.1, eq. 19, 23, 26-30)
    ("hrfd_normal_sign", "double n[3] = {0.0, (double)side, 0.0}, ni[3] = {0.0, (double)-side, 0.0};",
     "double n[3] = {0.0, (double)side, 0.0}, ni[3] = {0.0, (double)side, 0.0};", 1, "hrfd_cell or cai_degrigny_cell"),
    ("hrfd_fd_stencil_factor", "double g_fd = (-3.0 * ubwf + 4.0 * uF_t - uFF_t) / 2.0;",
     "double g_fd = (-3.0 * ubwf + 4.0 * uF_t - uFF_t);", 1, "hrfd_cell"),
    ("boundary_density_closure", "double rhoB = fpar + 2.0 * fperp;", "double rhoB = fpar + fperp;", 1,
     "boundary_density or hrfd_cell"),
    ("regularized_sign", "f[i] = feq[i] - w[i] * rho * tau / CS2 * QS;", "f[i] = feq[i] + w[i] * rho * tau / CS2 * QS;",
     1, "regularized_moments"),
    ("cai_degrigny_coefficient", "-11.0 / 6.0 * orc_uplus(law, yp, kappa, B)",
     "-11.0 / 5.0 * orc_uplus(law, yp, kappa, B)", 1, "cai_degrigny"),
    # flat-plate edges (Sec. 4.2.1)
    ("zou_he_sign", "f[5] = f[6] - 0.5 * (f[3] - f[4]) + (1.0 / 6.0) * rho * U;",
     "f[5] = f[6] + 0.5 * (f[3] - f[4]) + (1.0 / 6.0) * rho * U;", 1, "zou_he"),
    ("outlet_source_column", "if (o->c[3 * i] < 0) o->fnew[i * N + c1] = o->fnew[i * N + c2];",
     "if (o->c[3 * i] < 0) o->fnew[i * N + c1] = o->fnew[i * N + c1];", 1, "plate"),
]
