"""Mutation tests: plant plausible mistakes in the oracle's C source, rebuild
it on the CPU, and check that the pin suite (tests/test_oracle_pins.py)
fails for every one of them.  This shows the pins constrain each part of the
oracle: a dropped term, a wrong sign, a wrong index or a wrong order shows up.

Not listed: un-pinning s in the backward BFS.  Every solve saturates all of
s's out-arcs before its first global relabel and nothing refills them, so s
is never reachable there and that change is an equivalent mutant."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "clamp_wrong_sign": ("g->res[a ^ 1] += g->res[a];\n            g->res[a] = 0;",
                         "g->res[a ^ 1] -= g->res[a];\n            g->res[a] = 0;"),
    "deficits_not_seeded": ("if (v != g->s && v != g->t && g->e[v] < 0) {\n            g->h[v] = 0;",
                            "if (0) {\n            g->h[v] = 0;"),
    "value_drops_deficits": ("if (v != g->s && v != g->t && g->e[v] < 0) value += g->e[v];",
                             ";"),
    "no_resaturation_after_batch": ("    saturate_source(g);\n    /* 5.", "    /* 5."),
    "excess_recompute_sign": ("g->e[g->head[a]] += f;", "g->e[g->head[a]] -= f;"),
    "first_update_wins": ("        int64_t a = map_find(g, uu[i], vv[i]);\n        if (a < 0) a = new_arc_pair(g, uu[i], vv[i]);\n        g->res[a] += (int64_t)cc[i] - g->cap[a];",
                          "        int64_t a = map_find(g, uu[i], vv[i]);\n        if (a < 0) a = new_arc_pair(g, uu[i], vv[i]);\n        if (g->cap[a] != 0 && i > 0) { touched[i] = a; continue; }\n        g->res[a] += (int64_t)cc[i] - g->cap[a];"),
    "duplicates_not_summed": ("g->cap[a] += cap[i];", "g->cap[a] = cap[i];"),
    "ek_wrong_reverse_update": ("res[parent[v] ^ 1] += bottleneck;", "res[parent[v] ^ 1] += 0;"),
    "brute_cut_direction": ("if (in_s[src[i]] && !in_s[dst[i]]) c += cap[i];\n        if (best",
                            "if (!in_s[src[i]] && in_s[dst[i]]) c += cap[i];\n        if (best"),
    "bfs_uses_forward_residual": ("g->res[a ^ 1] > 0) {\n                g->h[w] = g->h[u] + 1;",
                                  "g->res[a] > 0) {\n                g->h[w] = g->h[u] + 1;"),
    "cert_skips_conservation": ("if (v != s && v != t && net[v] != 0) {", "if (0) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_kill_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    mut_c = tmp_path / "oracle_mut.c"
    mut_c.write_text(text.replace(old, new))
    mut_so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(mut_so),
                           str(mut_c)])
    env = dict(os.environ, MF_ORACLE_LIB=str(mut_so))
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert proc.returncode != 0, f"mutant {name} survived the pin suite:\n{proc.stdout[-2000:]}"
