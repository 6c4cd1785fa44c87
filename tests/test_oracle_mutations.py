"""Sensitivity of the oracle's pins: each plausible mistake planted in a copy
of the oracle (on the CPU) must make at least one pin fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_encode.py", "tests/test_oracle_distance.py", "tests/test_oracle_probe.py",
        "tests/test_oracle_graph.py", "tests/test_oracle_prune.py"]

MUTATIONS = {
    "round_half_even": ("float c = b + 0.5f;\n    float v = floorf(c);",
                        "float c = b;\n    float v = rintf(c);"),
    "no_clamp_top": ("if (v > (float)top) return top;", ""),
    "residual_step_pow2": ("delta2 = delta / (float)top2;", "delta2 = delta / (float)(top2 + 1u);"),
    "residual_wrong_offset": ("c2[j] = (uint8_t)quantize_one(r, -half, inv2, top2);",
                              "c2[j] = (uint8_t)quantize_one(r, 0.0f, inv2, top2);"),
    "turbo_transposed": ("dim = b * blk + 16 * k + w;", "dim = b * blk + per_word * w + k;"),
    "upper_bound_as_min": ("if (j == 0 || t[j] > u) u = t[j];", "if (j == 0 || t[j] < u) u = t[j];"),
    "full_level_sign": ("v += -0.5 * (double)delta", "v += 0.5 * (double)delta"),
    "mean_dropped": ("double v = (double)mu[j] + (double)l", "double v = (double)l"),
    "ties_to_highest_mean": ("if (m == 0 || s < best_s) {", "if (m == 0 || s <= best_s) {"),
    "topk_ties_reversed": ("return ia < ib;", "return ia > ib;"),
    "nibble_order": ("return (codes[p / 2] >> (4 * (p % 2))) & 0xFu;",
                     "return (codes[p / 2] >> (4 * (1 - p % 2))) & 0xFu;"),
    "step_off_by_one": ("delta = (u - l) / (float)top1;", "delta = (u - l) / (float)(top1 + 1u);"),
    "probe_ties_to_higher_mean": ("return ma < mb;", "return ma > mb;"),
    "probe_nan_first": ("if (isnan(sa) != isnan(sb)) return isnan(sb);", "if (isnan(sa) != isnan(sb)) return isnan(sa);"),
    "probe_distance_unsquared": ("float sq = e * e;", "float sq = fabsf(e);"),
    "eps1_per_vector_mean": ("    free(xhat);\n    return total;\n}", "    free(xhat);\n    return total / (double)n;\n}"),
    "eps1_absolute_error": ("            total += e * e;", "            total += fabs(e);"),
}

# mistakes in the graph functions of oracle/__init__.py (Alg. 1, Alg. 2, App. A)
PY_MUTATIONS = {
    "prune_rule_reversed_l2": ("removed = alpha * t <= sims[c] if metric == L2",
                               "removed = alpha * t >= sims[c] if metric == L2"),
    "prune_alpha_on_node_side": ("removed = alpha * t <= sims[c] if metric == L2",
                                 "removed = t <= alpha * sims[c] if metric == L2"),
    "prune_rule_reversed_ip": ("else alpha * t >= sims[c]", "else alpha * t <= sims[c]"),
    "prune_keeps_node": ("for c in list(cand) + list(current) if c >= 0) - {int(p)})",
                         "for c in list(cand) + list(current) if c >= 0))"),
    "prune_ignores_current": ("for c in list(cand) + list(current) if c >= 0)",
                              "for c in list(cand) if c >= 0)"),
    "prune_ties_to_higher": ("key=lambda c: (sims[c] if metric == L2 else -sims[c], c))",
                             "key=lambda c: (sims[c] if metric == L2 else -sims[c], -c))"),
    "walk_cut_off_by_one": ("cand = dict(ranked[:W])", "cand = dict(ranked[:W + 1])"),
    "walk_explores_worst": ("x = open_[0][0]", "x = open_[-1][0]"),
    "walk_returns_deleted": ("if live is None or live[it[0]]]", "]"),
    "insert_no_reverse_edges": ("        for y in nx:\n            ny = row(y)\n", "        for y in []:\n            ny = row(y)\n"),
    "batched_first_pass_unbounded": ("bs = min(B, max(1, now), count - b)", "bs = min(B, count - b)"),
    "batched_overflow_truncated": ("                    put(y, robust_prune(metric, X, y, S, ny, a, R))",
                                   "                    put(y, union[:R])"),
    "batched_second_pass_alpha_one": ("a = 1.0 if (passes == 2 and pass_ == 0) else alpha", "a = 1.0"),
    "delete_rows_kept": ("    out[deleted] = -1\n    return out", "    return out"),
    "delete_never_prunes": ("if len(cand) > R else cand", "if False else cand"),
    "recall_counts_repeats": ("hits = sum(len(set(found[i].tolist()) & set(truth[i].tolist()))",
                              "hits = sum(sum(int(v in set(truth[i].tolist())) for v in found[i].tolist())"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS) + sorted(PY_MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    target = "lvq_oracle.c" if name in MUTATIONS else "__init__.py"
    old, new = MUTATIONS[name] if name in MUTATIONS else PY_MUTATIONS[name]
    work = tmp_path / "repo"
    (work / "tests").mkdir(parents=True)
    shutil.copytree(os.path.join(ROOT, "oracle"), work / "oracle",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "synth"), work / "synth",
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), work / "tests" / "golden")
    for f in PINS + ["tests/conftest.py"]:
        shutil.copy(os.path.join(ROOT, f), work / f)
    src = work / "oracle" / target
    text = src.read_text()
    assert text.count(old) == 1, "mutation anchor not found: " + name
    src.write_text(text.replace(old, new))
    env = dict(os.environ, PYTHONPATH=str(work), PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=work, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])
