"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the
CPU), builds it, and runs the pin tests against that build in a child
process; every mutant must make at least one pin fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lcd_oracle.c")

MUTANTS = {
    "k_in_single_count": ("g->K += 2 * g->d[u];\n    g->V += g->k[u];\n    g->size += 1;\n    g->M += 1;",
                          "g->K += g->d[u];\n    g->V += g->k[u];\n    g->size += 1;\n    g->M += 1;"),
    "removal_single_count": ("g->K -= 2 * g->d[u];", "g->K -= g->d[u];"),
    "alpha_on_wrong_log": ("double c = alpha * lcdo_log((uint64_t)k);\n    return lcdo_log((uint64_t)(2 * d)) - c;",
                           "double c = alpha * lcdo_log((uint64_t)(2 * d));\n    return c - lcdo_log((uint64_t)k);"),
    "tie_larger_id_first": ("(a->r == b->r && a->u < b->u)", "(a->r == b->r && a->u > b->u)"),
    "criterion_sign": ("double t = a - c;", "double t = a + c;"),
    "no_requeue_after_reject": ("        if (!g->in_c[v])\n            lcdo_queue(g, v, alpha);",
                                "        if (!g->in_c[v] && g->queued[v])\n            lcdo_queue(g, v, alpha);"),
    "prune_descending": ("return (x > y) - (x < y);", "return (x < y) - (x > y);"),
    "no_prune": ("    if (added) {\n        for (uint32_t pass", "    if (0 && added) {\n        for (uint32_t pass"),
    "volume_misses_new_node": ("g->V += g->k[u];\n    g->size += 1;\n    g->M += 1;",
                               "g->size += 1;\n    g->M += 1;"),
    "margin_dropped": ("return t > 0x1p-40;", "return t >= 0.0;"),
    "seed_candidates_degree_one": ("cand[u] = (g->row_ptr[u + 1] - g->row_ptr[u]) >= 2;",
                                   "cand[u] = (g->row_ptr[u + 1] - g->row_ptr[u]) >= 1;"),
    "seed_rule2_one_hop": ("            if (rule == 2)\n                for (int64_t q",
                           "            if (rule == 3)\n                for (int64_t q"),
    "merge_survivor_higher_id": ("                        m.alive[b] = 0;\n                        m.into[b] = a;\n                        need[a] = 1;",
                                 "                        m.alive[b] = 0;\n                        m.into[b] = a;\n                        need[a] = 1;\n                        { int32_t *t_ = m.mem[a]; m.mem[a] = m.mem[b]; m.mem[b] = t_; }"),
    "merge_threshold_uses_larger": ("const int64_t small = m->msz[c] < m->msz[i] ? m->msz[c] : m->msz[i];",
                                    "const int64_t small = m->msz[c] > m->msz[i] ? m->msz[c] : m->msz[i];"),
    "merge_growth_to_fixpoint": [("&alpha, 1, k_prune, 1, tmp, n, off2, &k1,", "&alpha, 1, k_prune, 0, tmp, n, off2, &k1,"),
                                 ("need[j] = changed[j];", "need[j] = 0;")],
    "nmi_admission_reversed": ("if (!(ha + he > hb + hc))", "if (!(ha + he < hb + hc))"),
    "nmi_max_instead_of_min": ("if (!found || cond < best) {", "if (!found || cond > best) {"),
    "nmi_unnormalised": ("sum += best / hx;", "sum += best;"),
    "nmi_joint_drops_a_cell": ("const double hxy = ((ha + hb) + hc) + he;", "const double hxy = (ha + hb) + hc;"),
    "rank_uses_d_out": ("lcdo_push(g, lcdo_rank(g->d[u], g->k[u], alpha), u, g->ver[u]);",
                        "lcdo_push(g, lcdo_rank(g->d[u], g->k[u] - g->d[u] + 1, alpha), u, g->ver[u]);"),
}

PINS = ["tests/test_oracle_bruteforce.py", "tests/test_oracle_replay.py",
        "tests/test_oracle_limits.py", "tests/test_oracle_audit.py"]
# mutants of the seed selection and of the merge phase are run against the
# pins of that part only
PINS_OF = {"seed_": ["tests/test_oracle_seeds.py"], "merge_": ["tests/test_oracle_merge.py"],
           "nmi_": ["tests/test_oracle_nmi.py"]}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    edits = MUTANTS[name]
    if isinstance(edits, tuple):
        edits = [edits]
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    mut = tmp_path / "mutant.c"
    mut.write_text(src)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                    str(mut), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, LCDO_LIB=str(so))
    # a mutant that makes the growth loop run away is caught by the per-test
    # time limit (the thread method also stops a hang inside the C code)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "--timeout", "20", "--timeout-method", "thread",
                        *next((v for k, v in PINS_OF.items() if name.startswith(k)), PINS)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode != 0, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])
