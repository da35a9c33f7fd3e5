"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, a swapped operand
or index) in a copy of the oracle's C source, builds it on the CPU, and runs
the pin tests against the broken copy in a subprocess: at least one pin must
fail.  Nothing here touches the GPU or the HIP library.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hydro_oracle.c")

MUTATIONS = {
    "eos_drops_kinetic": ("(gamma - 1.0) * (U[4] - kinetic)", "(gamma - 1.0) * (U[4])"),
    "limiter_drops_factor_2": ("(2.0 * prod) / (dl + dr)", "prod / (dl + dr)"),
    "predictor_sign": ("Wt[v] = Wc[v] - 0.5 *", "Wt[v] = Wc[v] + 0.5 *"),
    "predictor_drops_dp_over_rho": ("out[1 + d] += dW[4] / rho;", ""),
    "predictor_drops_gamma": ("out[4] = gamma * p * dW[1 + d]", "out[4] = p * dW[1 + d]"),
    "predictor_tangential_uses_normal": ("out[2] = un * dW[2];", "out[2] = un * dW[1];"),
    "face_state_sign": ("Wp[5 * mL + v] + 0.5 * S", "Wp[5 * mL + v] - 0.5 * S"),
    "face_state_wrong_direction": ("S[15 * mR + 5 * d + v]", "S[15 * mR + 5 * ((d + 1) % 3) + v]"),
    "davis_speed_swapped": ("(uL - cL < uR - cR) ? uL - cL : uR - cR", "(uL - cL < uR - cR) ? uR - cR : uL - cL"),
    "star_energy_sign": ("(Sstar + p / (rho * (S - un)))", "(Sstar - p / (rho * (S - un)))"),
    "star_tangential_dropped": ("Us[2] = factor * W[2];", "Us[2] = factor;"),
    "energy_flux_drops_p": ("F[4] = un * (E + W[4]);", "F[4] = un * E;"),
    "update_sign": ("Un[v] = Ub[at(g, v, i, j, k)] - div;\n          if (U0b)",
                    "Un[v] = Ub[at(g, v, i, j, k)] + div;\n          if (U0b)"),
    "ctu_update_sign": ("Un[v] = Ub[at(g, v, i, j, k)] - div;\n          Uo[at(g, v, i, j, k)] = Un[v];\n        }\n        int ok",
                        "Un[v] = Ub[at(g, v, i, j, k)] + div;\n          Uo[at(g, v, i, j, k)] = Un[v];\n        }\n        int ok"),
    "lambda_z_uses_dy": ("dt / g->dx[2]};\n  const size_t bd = oracle_block_doubles(g);\n  const double *Ub = U + (size_t)b * bd;\n  /* Cells that need",
                         "dt / g->dx[1]};\n  const size_t bd = oracle_block_doubles(g);\n  const double *Ub = U + (size_t)b * bd;\n  /* Cells that need"),
    "ctu_lambda_z_uses_dy": ("dt / g->dx[2]};\n  const size_t bd = oracle_block_doubles(g);\n  const double *Ub = U + (size_t)b * bd;\n  const int m",
                             "dt / g->dx[1]};\n  const size_t bd = oracle_block_doubles(g);\n  const double *Ub = U + (size_t)b * bd;\n  const int m"),
    "outflow_clamp_wrong_end": ("if (I > N - 1) return N - 1;", "if (I > N - 1) return N - 2;"),
    "periodic_wrap_off_by_one": ("return r < 0 ? r + N : r;", "return r < 0 ? r + N - 1 : r;"),
    "dt_drops_sound_speed_in_z": ("(fabs(W[3]) + c) / g->dx[2]", "fabs(W[3]) / g->dx[2]"),
    "fallback_never_applies": ("if (!(r > 0.0) || !(p > 0.0)) bad = 1;", ""),
    "rk2_final_weights": ("stage_all(g, U1, U, 0.5, 0.5, Unew, dt, cnt);", "stage_all(g, U1, U, 0.0, 1.0, Unew, dt, cnt);"),
    "rk3_middle_weights": ("stage_all(g, U1, U, 0.75, 0.25, U2, dt, cnt);", "stage_all(g, U1, U, 0.25, 0.75, U2, dt, cnt);"),
    "rk3_final_input": ("stage_all(g, U2, U, 1.0 / 3.0, 2.0 / 3.0, Unew, dt, cnt);",
                        "stage_all(g, U1, U, 1.0 / 3.0, 2.0 / 3.0, Unew, dt, cnt);"),
    "stage_weights_swapped": ("Un[v] = a0 * U0b[at(g, v, i, j, k)] + a1 * Un[v];",
                              "Un[v] = a1 * U0b[at(g, v, i, j, k)] + a0 * Un[v];"),
    "stage_uses_predictor": ("Uo + (size_t)b * bd, dt, 0,", "Uo + (size_t)b * bd, dt, 1,"),
    "stage_skips_guard_fill": ("oracle_fill_guards(g, Us);", ""),
    "ctu_corner_weight_half": ("(lam[t] / 3.0)", "(lam[t] / 2.0)"),
    "ctu_final_weight_one": ("0.5 * (lam[t] * (Fc[", "1.0 * (lam[t] * (Fc["),
    "ctu_final_cross_index": ("const int kt = tr[t][0] == u ? 0 : 1;", "const int kt = tr[t][0] == u ? 1 : 0;"),
    "ctu_corner_uses_own_direction": ("(F1[15 * ch + 5 * t + v] - F1[15 * cc + 5 * t + v])",
                                      "(F1[15 * ch + 5 * d + v] - F1[15 * cc + 5 * d + v])"),
    "ctu_trace_acoustic_sign": ("const double bm = 0.5 * (S[4] / (c * c) - rho * S[1 + d] / c);",
                                "const double bm = 0.5 * (S[4] / (c * c) + rho * S[1 + d] / c);"),
    "ctu_trace_courant_sign": ("hi[v] += 0.5 * (1.0 - lam * speed[k]) * wave[k][v];",
                               "hi[v] += 0.5 * (1.0 + lam * speed[k]) * wave[k][v];"),
    "ctu_trace_entropy_drops_dp": ("wave[1][0] = S[0] - S[4] / (c * c);", "wave[1][0] = S[0];"),
    "ctu_trace_normal_eigvec_sign": ("wave[2][1 + d] = bp * c / rho;", "wave[2][1 + d] = -bp * c / rho;"),
    "ctu_trace_keeps_waves_moving_away": ("    if (speed[k] < 0.0)\n      for (int v = 0; v < 5; ++v) lo[v]",
                                          "    if (speed[k] != 0.0)\n      for (int v = 0; v < 5; ++v) lo[v]"),
    "ctu_dt_sums_directions": ("else if (s > smax) smax = s;\n          }\n        }\n  }\n  return bad ? NAN : smax;\n}\n\ndouble oracle_dt_ctu",
                               "else if (s > smax) smax = s;\n          }\n        }\n  }\n  return bad ? NAN : 3.0 * smax;\n}\n\ndouble oracle_dt_ctu"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    mut = tmp_path / "hydro_oracle.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "hydro_oracle.h")
    (tmp_path / "hydro_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-std=c99", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, HYDRO_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    # a mistake in a scheme-specific path is looked for by that scheme's pins
    # first (the suite stops at the first failure either way)
    files = ["tests/test_oracle_units.py", "tests/test_oracle_step.py", "tests/test_oracle_fallback.py",
             "tests/test_oracle_rk.py", "tests/test_oracle_ctu.py"]
    first = {"ctu": "tests/test_oracle_ctu.py", "rk": "tests/test_oracle_rk.py",
             "stage": "tests/test_oracle_rk.py"}.get(name.split("_")[0])
    if first:
        files.remove(first)
        files.insert(0, first)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived all pins:\n{r.stdout[-2000:]}"


# Mistakes planted in the two-level AMR step (oracle/amr.py, numpy).
AMR_MUTATIONS = {
    "amr_no_reflux": ("corr = lam0[d] * (Fc - Ff) * (1.0 if side else -1.0)",
                      "corr = 0.0 * lam0[d] * (Fc - Ff) * (1.0 if side else -1.0)"),
    "amr_reflux_sign": ("corr = lam0[d] * (Fc - Ff) * (1.0 if side else -1.0)",
                        "corr = lam0[d] * (Fc - Ff) * (-1.0 if side else 1.0)"),
    "amr_reflux_wrong_face": ("Fc = _face(flux0[b][d], d, n, n if side else 0)",
                              "Fc = _face(flux0[b][d], d, n, 0 if side else n)"),
    "amr_prolong_slope_sign": ("val = val + S * (0.25 * offs[d])", "val = val - S * (0.25 * offs[d])"),
    "amr_prolong_half_weight": ("val = val + S * (0.25 * offs[d])", "val = val + S * (0.5 * offs[d])"),
    "amr_indicator_num_sign": ("num = (fR - f) - (f - fL)", "num = (fR - f) + (f - fL)"),
    "amr_indicator_den_no_abs": ("den = (np.abs(fR - f) + np.abs(f - fL))", "den = ((fR - f) + (f - fL))"),
    "amr_indicator_density_only": ("E2 = np.maximum(_second_difference_ratio(mesh, rho, eps), "
                                   "_second_difference_ratio(mesh, p, eps))",
                                   "E2 = np.maximum(_second_difference_ratio(mesh, rho, eps), "
                                   "_second_difference_ratio(mesh, rho, eps))"),
    "amr_flags_no_derefine": ("new[mesh.refine & (E2 < derefine_cutoff * derefine_cutoff)] = False",
                              "new[mesh.refine & (E2 < derefine_cutoff * derefine_cutoff)] = True"),
    "amr_regrid_injects": ("Uf2[f] = prolong(new, Ur, I.ravel(), J.ravel(), K.ravel()).reshape(5, n, n, n)",
                           "Uf2[f] = root_value(new, Ur, I.ravel() // 2, J.ravel() // 2, K.ravel() // 2)"
                           ".reshape(5, n, n, n)"),
    "amr_regrid_wrong_child_kept": ("Uf2[f] = Uf[int(mesh.child_base[r]) + c]",
                                    "Uf2[f] = Uf[int(mesh.child_base[r]) + (c ^ 1)]"),
    "amr_restrict_wrong_child": ("cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1\n            ch = Uf[8 * q + c]",
                                 "cx, cy, cz = (c >> 1) & 1, c & 1, (c >> 2) & 1\n            ch = Uf[8 * q + c]"),
}


# Mistakes planted in the oracle's AMR of any depth (oracle/amr_tree.py).
TREE_MUTATIONS = {
    "tree_restrict_top_down": ("for l in range(t.levels - 2, -1, -1):", "for l in range(t.levels - 1):"),
    "tree_prolong_same_level": ("Uc = level_value(t, U, l - 1, Ic, Jc, Kc)",
                                "Uc = level_value(t, U, l - 1, Ic, Jc, Kc) * (1.0 + 1e-3)"),
    "tree_reflux_wrong_level_dx": ("lam = [dt / h for h in t.dx(l)]", "lam = [dt / h for h in t.dx(l + 1)]"),
    "tree_no_nesting_repair": ("    changed = True\n    while changed:\n        changed = False\n        # drop",
                               "    changed = False\n    while changed:\n        changed = False\n        # drop"),
    "tree_indicator_missing_is_zero": ("u[:, ~ok] = own[:, ~ok]", "u[:, ~ok] = 0.0 * own[:, ~ok]"),
    "tree_regrid_injects": ("Ul[i] = prolong(new, V, l, I.ravel(), J.ravel(), K.ravel()).reshape(5, n, n, n)",
                            "Ul[i] = level_value(new, V, l - 1, I.ravel() // 2, J.ravel() // 2, K.ravel() // 2)"
                            ".reshape(5, n, n, n)"),
    "tree_copy_from_parent_level": ("out[:, here] = U[l][blk[here], :, K[here] % n, J[here] % n, I[here] % n].T",
                                    "out[:, here] = U[l][blk[here], :, K[here] % n, J[here] % n, I[here] % n].T"
                                    " * (1.0 + 1e-12 * (l > 1))"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(TREE_MUTATIONS))
def test_tree_pins_catch_planted_mistake(name, tmp_path):
    import shutil

    old, new = TREE_MUTATIONS[name]
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (pkg / "amr_tree.py").read_text()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    (pkg / "amr_tree.py").write_text(src.replace(old, new))
    import oracle

    shutil.copy(os.path.join(ROOT, "tests", "test_oracle_amr_tree.py"), tmp_path / "test_oracle_amr_tree.py")
    os.makedirs(tmp_path / "tests", exist_ok=True)
    (tmp_path / "tests" / "__init__.py").write_text("")
    shutil.copy(os.path.join(ROOT, "tests", "test_oracle_amr.py"), tmp_path / "tests" / "test_oracle_amr.py")
    env = dict(os.environ, HYDRO_ORACLE_LIB=oracle.LIB_PATH, OMP_NUM_THREADS="4",
               PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT, os.environ.get("PYTHONPATH", "")]))
    probe = subprocess.run([sys.executable, "-c", "import oracle.amr_tree as a; print(a.__file__)"], cwd=tmp_path,
                           env=env, capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().startswith(str(tmp_path)), probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "test_oracle_amr_tree.py"], cwd=tmp_path, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, f"mutation {name} survived the tree pins:\n{r.stdout[-2000:]}"


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(AMR_MUTATIONS))
def test_amr_pins_catch_planted_mistake(name, tmp_path):
    import shutil

    old, new = AMR_MUTATIONS[name]
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (pkg / "amr.py").read_text()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    (pkg / "amr.py").write_text(src.replace(old, new))
    import oracle

    # run the pins from a directory of their own so that `import oracle`
    # finds the mutated copy first (the rest comes from the repository)
    shutil.copy(os.path.join(ROOT, "tests", "test_oracle_amr.py"), tmp_path / "test_oracle_amr.py")
    env = dict(os.environ, HYDRO_ORACLE_LIB=oracle.LIB_PATH, OMP_NUM_THREADS="4",
               PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT, os.environ.get("PYTHONPATH", "")]))
    probe = subprocess.run([sys.executable, "-c", "import oracle.amr as a; print(a.__file__)"], cwd=tmp_path,
                           env=env, capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().startswith(str(tmp_path)), probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "test_oracle_amr.py"], cwd=tmp_path, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, f"mutation {name} survived the AMR pins:\n{r.stdout[-2000:]}"
