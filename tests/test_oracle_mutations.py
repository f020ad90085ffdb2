"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the
pins catch every one: a dropped term, a wrong sign or index, a transposed
scaling, a non-strict cutoff, a wrong quantization, a wrong Philox constant,
a pre-pass that ignores the diagonal's sign, uses another norm or cuts at the
wrong rank, a top-k selection that keeps the wrong number or the wrong end, row
features with the wrong weighting, an allocation that truncates, a Neyman
target without its square root, an Adam step without bias correction.
Mutations name the file of the oracle they change (mcmi_oracle.c by default)."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "drop_j0_term": ("        double w = 1.0;\n        visit(ctx, s, w);", "        double w = 1.0;\n"),
    "ignore_sign": ("            w = (A->cval[k] < 0.0) ? -wn : wn;\n            s = A->ccol[k];\n            visit(ctx, s, w);\n            ++steps;\n        }\n    } else {",
                    "            w = wn;\n            s = A->ccol[k];\n            visit(ctx, s, w);\n            ++steps;\n        }\n    } else {"),
    "scale_by_row_diag": ("double m = nhat / A->diag[col];", "double m = nhat / A->diag[r];"),
    "cutoff_not_strict": ("if (fabs(wn) < p->delta)", "if (fabs(wn) <= p->delta)"),
    "quantize_ceil": ("double scaled = floor(ldexp(ratio, q));", "double scaled = ceil(ldexp(ratio, q));"),
    "alias_threshold_inclusive": ("if (r < (uint64_t)A->athr[b + (int64_t)j])",
                                  "if (r <= (uint64_t)A->athr[b + (int64_t)j])"),
    "alias_gives_away_too_much": ("q[lg] -= W - q[sm];", "q[lg] -= W;"),
    "alias_bucket_off_by_one": ("uint64_t j = um >> 32;", "uint64_t j = ((uint64_t)u * (m - 1)) >> 32;"),
    "shat_is_amax": ("shat[i] = ldexp(amax * (double)run, -q);", "shat[i] = amax;"),
    "philox_multiplier": ("0xD2511F53u", "0xD2511F55u"),
    "near_cutoff_band_per_step_missing": ("return fabs(a - delta) <= (2.0 * (double)j + 1.0) * u32",
                                          "return fabs(a - delta) <= u32"),
    "near_cutoff_not_counted": ("                border += near;", "                border += 0 * near;"),
    "aug_ignores_sign": ("d = d + (d < 0.0 ? -aug : aug);", "d = d + aug;"),
    "aug_norm_is_max_entry": ("s += fabs(v[k]);", "s = fabs(v[k]) > s ? fabs(v[k]) : s;"),
    "drop_cut_off_by_one": ("thr = mag[K];", "thr = mag[K > 0 ? K - 1 : 0];"),
    "drop_keeps_ties_out": ("if (fabs(c) < thr) {", "if (fabs(c) <= thr && thr > 0.0) {"),
    "topk_ignores_diagonal_slot": ("int64_t want = (int64_t)p->topk - 1;", "int64_t want = (int64_t)p->topk;"),
    "topk_keeps_smallest": ("return x->test > y->test ? -1 : 1;", "return x->test < y->test ? -1 : 1;"),
    "features_uniform_weights": ("double pk = (double)w / (double)A->wsum[i];", "double pk = 1.0 / (double)m;"),
    "features_sign_balance_of_magnitudes": ("csum += A->cval[k] < 0.0 ? -chat : chat;", "csum += chat;"),
    "features_max_of_weights": ("if (chat > cmax)\n                cmax = chat;",
                                "if (pk > cmax)\n                cmax = pk;"),
    "alloc_truncates": ("ref.py", "n_r = np.maximum(1, np.rint(lam * e)).astype(np.int64)",
                        "n_r = np.maximum(1, np.floor(lam * e)).astype(np.int64)"),
    "neyman_without_sqrt": ("ref.py", "return 0.5 * (np.log(v) - np.log(np.asarray(mean_len, dtype=np.float64) + 1.0))",
                            "return np.log(v) - np.log(np.asarray(mean_len, dtype=np.float64) + 1.0)"),
    "neyman_cost_without_start": ("ref.py",
                                  "return 0.5 * (np.log(v) - np.log(np.asarray(mean_len, dtype=np.float64) + 1.0))",
                                  "return 0.5 * (np.log(v) - np.log(np.asarray(mean_len, dtype=np.float64) + 1e-300))"),
    "chain_cost_ceiling": ("ref.py", "return (1 + np.floor(np.maximum(f, 0.0))).astype(np.int64)",
                           "return (1 + np.ceil(np.maximum(f, 0.0))).astype(np.int64)"),
    "adam_no_bias_correction": ("ref.py", "mh = m / (1 - beta1 ** t)", "mh = m"),
    "adam_second_moment_of_abs": ("ref.py", "v[...] = beta2 * v + (1 - beta2) * g[name] * g[name]",
                                  "v[...] = beta2 * v + (1 - beta2) * np.abs(g[name])"),
}

DRIVER = textwrap.dedent('''
    import importlib.util, sys, traceback, os, shutil, subprocess, tempfile
    sys.path.insert(0, sys.argv[1])   # the mutated oracle first
    sys.path.insert(1, sys.argv[2])   # the repository (inputs)
    import oracle
    oracle.build(force=True)
    spec = importlib.util.spec_from_file_location("pins", os.path.join(sys.argv[2], "tests", "test_oracle_pins.py"))
    pins = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(pins)
    calls = [
        ("p1", lambda: pins.test_p1_diagonal_matrix_gives_exact_inverse_and_no_transitions()),
        ("p2_nil", lambda: pins.test_p2_nilpotent_shift_equals_triangular_solve()),
        ("p2_cyc", lambda: pins.test_p2_scaled_cycle_closed_form(-0.7)),
        ("p3", lambda: pins.test_p3_torus_row_sums_and_exact_transition_count()),
        ("p5", lambda: pins.test_p5_converges_to_numpy_inverse(1)),
        ("p6", lambda: pins.test_p6_matches_exact_rational_expectation("tiny3_signed")),
        ("quant", lambda: pins.test_cdf_quantization_bounds()),
        ("quant_exact", lambda: pins.test_integer_weights_are_exact_floors()),
        ("strict", lambda: pins.test_cutoff_is_strict_when_weight_equals_delta()),
        ("alias_mass", lambda: pins.test_alias_tables_conserve_every_entry_mass()),
        ("alias_draw", lambda: pins.test_alias_draw_probabilities_and_boundaries()),
        ("aug", lambda: pins.test_augmented_splitting_equals_the_hand_built_matrix()),
        ("reduce", lambda: pins.test_reduction_drops_the_smallest_share_of_the_iteration_matrix()),
        ("compose", lambda: pins.test_augmentation_then_reduction_compose()),
        ("topk", lambda: pins.test_topk_keeps_the_largest_entries_of_the_eps_set()),
        ("features", lambda: pins.test_features_of_a_hand_built_matrix()),
        ("alloc_unit", lambda: pins.test_allocation_lambda_by_hand("unit_cost")),
        ("alloc_floor", lambda: pins.test_allocation_lambda_by_hand("floor_of_one")),
        ("neyman", lambda: pins.test_neyman_target_gives_the_brute_force_optimum()),
        ("adam", lambda: pins.test_adam_two_steps_by_hand()),
        ("cost", lambda: pins.test_chain_cost_counts_the_states_of_every_chain("uniform_0.7")),
        ("near0", lambda: pins.test_near_cutoff_count_is_zero_far_from_delta()),
        ("near1", lambda: pins.test_near_cutoff_count_at_a_weight_equal_or_next_to_delta(1.0e-6, True, 9)),
        ("near3", lambda: pins.test_near_cutoff_count_at_a_weight_equal_or_next_to_delta(3.0e-6, False, 9)),
    ]
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if os.path.exists(hipcc):
        d = tempfile.mkdtemp()
        src = os.path.join(d, "rr.cpp")
        open(src, "w").write(pins.ROCRAND_PROBE)
        exe = os.path.join(d, "rr")
        if subprocess.call([hipcc, "-O1", "-o", exe, src], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL) == 0:
            calls.append(("p12", lambda: pins.test_p12_philox_matches_rocrand(exe)))
    failed = []
    for name, fn in calls:
        try:
            fn()
        except Exception:
            failed.append(name)
    print("FAILED:" + ",".join(failed))
''')


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    mut = MUTATIONS[name]
    fname, old, new = mut if len(mut) == 3 else ("mcmi_oracle.c",) + mut
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (dst / fname).read_text()
    assert src.count(old) >= 1, "mutation anchor not found"
    (dst / fname).write_text(src.replace(old, new, 1))
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    out = subprocess.run([sys.executable, str(drv), str(tmp_path), ROOT], capture_output=True, text=True,
                         timeout=600)
    line = [l for l in out.stdout.splitlines() if l.startswith("FAILED:")]
    assert line, out.stdout[-2000:] + out.stderr[-2000:]
    caught = [x for x in line[-1][len("FAILED:"):].split(",") if x]
    print(f"{name}: caught by {caught}")
    assert caught, f"mutation {name} passed every pin"


def test_unmutated_oracle_passes_the_driver(tmp_path):
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    out = subprocess.run([sys.executable, str(drv), str(tmp_path), ROOT], capture_output=True, text=True,
                         timeout=600)
    assert "FAILED:" in out.stdout and out.stdout.strip().splitlines()[-1] == "FAILED:", out.stdout[-2000:]
