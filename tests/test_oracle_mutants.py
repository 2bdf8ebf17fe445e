"""Shows that the oracle's pins have teeth: each case plants one plausible
mistake in a private copy of the C oracle (CPU only), builds it, and runs the
pin suite against it; the suite must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "kz_oracle.c")
EXT = os.path.join(ROOT, "oracle", "kz_oracle_ext.c")

MUTANTS = {
    "edge_threshold_k_minus_1": (
        "ci_edge(g, u, v, g->k - 2) < g->k - 2", "ci_edge(g, u, v, g->k - 1) < g->k - 1"),
    "vertex_threshold_k_minus_2": (
        "ci_vertex(g, v, g->k - 1) < g->k - 1", "ci_vertex(g, v, g->k - 2) < g->k - 2"),
    "edge_index_ignores_second_endpoint": (
        "if (edge_alive(g, v, w)) { g->stamp[c] = g->stamp_now; ++count; }",
        "if (1) { g->stamp[c] = g->stamp_now; ++count; }"),
    "edge_index_uses_endpoint_colour": (
        "    int32_t w = g->nb[e];\n    int32_t c = g->col[w];",
        "    int32_t w = g->nb[e];\n    int32_t c = g->col[u];"),
    "removals_applied_inside_the_round": (
        "if (u < v && g->ea[e] && edge_fails(g, u, v)) { fe[e] = 1; any = 1; }",
        "if (u < v && g->ea[e] && edge_fails(g, u, v)) { fe[e] = 1; any = 1; kill_entry(g, e); }"),
    "rounds_count_the_confirming_pass": ("stats[0] = rounds;", "stats[0] = rounds + 1;"),
    "failing_edge_output_stuck_at_zero": (
        "efail[i] = edge_alive(g, us[i], ws[i]) && edge_fails(g, us[i], ws[i]);", "efail[i] = 0;"),
    "o3_edge_test_skips_only_one_endpoint_class": (
        "            if (c == col[u] || c == cv) continue;", "            if (c == col[u]) continue;"),
    "o3_failed_edge_cleared_during_the_scan": (
        "          if (miss > slack) { fu[w] |= 1ull << j; any = 1; }",
        "          if (miss > slack) { fu[w] |= 1ull << j; any = 1; ((uint64_t *)ru)[w] &= ~(1ull << j); }"),
    "o3_vertex_test_skips_the_last_class": (
        "      for (int32_t c = 0; c < k && miss <= slack; ++c) {\n        if (c == col[v]) continue;",
        "      for (int32_t c = 0; c < k - 1 && miss <= slack; ++c) {\n        if (c == col[v]) continue;"),
    "o3_vertex_slack_ignored": ("      fv[v] = miss > slack;", "      fv[v] = miss > 0;"),
    "o3_edge_slack_off_by_one": (
        "          if (miss > slack) { fu[w] |= 1ull << j; any = 1; }",
        "          if (miss >= slack && miss) { fu[w] |= 1ull << j; any = 1; }"),
    "o3_rounds_count_the_confirming_pass": ("{rounds, rounds == 0,", "{rounds + 1, rounds == 0,"),
    "set_masks_accepts_one_way_edges": (
        "    if (g->ea[e] != g->ea[g->mate[e]]) return -1;\n", ""),
    "set_masks_ignores_dead_endpoints": (
        "    if (g->ea[e] && (!g->va[g->src[e]] || !g->va[g->nb[e]])) return -1;\n", ""),
    "vertex_index_counts_removed_edges": (
        "  for (int64_t e = g->rp[v]; e < g->rp[v + 1] && count < cap; ++e) {\n    if (!g->ea[e]) continue;",
        "  for (int64_t e = g->rp[v]; e < g->rp[v + 1] && count < cap; ++e) {\n    if (0) continue;"),
}


# Mistakes planted in kz_oracle_ext.c (dominance, clique search, struction,
# colourings); its pins are tests/test_oracle_ext.py.
EXT_MUTANTS = {
    "jp_takes_the_smallest_key": (
        "  return pri[u] > pri[v] || (pri[u] == pri[v] && u > v);",
        "  return pri[u] < pri[v] || (pri[u] == pri[v] && u < v);"),
    "jp_no_tie_break_by_index": (
        "  return pri[u] > pri[v] || (pri[u] == pri[v] && u > v);", "  return pri[u] > pri[v];"),
    "jp_colour_above_the_largest_used": (
        "      while (used[c]) ++c;", "      for (int32_t x = 0; x <= n; ++x) if (used[x]) c = x + 1;"),
    "jp_coloured_neighbours_block": (
        "if (adj[(int64_t)v * n + u] && colour[u] < 0 && jp_beats(pri, u, v)) best = 0;",
        "if (adj[(int64_t)v * n + u] && jp_beats(pri, u, v)) best = 0;"),
    "dom_vertex_subset_reversed": (
        "    if (adj[(int64_t)a * n + x] && !adj[(int64_t)b * n + x]) return 0;",
        "    if (adj[(int64_t)b * n + x] && !adj[(int64_t)a * n + x]) return 0;"),
    "dom_vertex_only_later_nodes": (
        "      for (int32_t a = 0; a < n; ++a) {\n        if (vertex_dominates",
        "      for (int32_t a = b + 1; a < n; ++a) {\n        if (vertex_dominates"),
    "dom_vertex_edges_left_at_the_neighbours": (
        "      adj[(int64_t)x * n + a] = 0;\n      ++removed;", "      ++removed;"),
    "dom_vertex_single_sweep": ("    if (!any) break;\n    ++sweeps;\n  }\n  stats[0] = sweeps;\n  stats[1] = dv;",
                                "    break;\n  }\n  stats[0] = sweeps;\n  stats[1] = dv;"),
    "dom_edge_whole_neighbourhood": (
        "    if (adj[(int64_t)a * n + x] && adj[(int64_t)u * n + x] && !adj[(int64_t)b * n + x]) return 0;",
        "    if (adj[(int64_t)a * n + x] && !adj[(int64_t)b * n + x]) return 0;"),
    "dom_edge_one_direction": ("            adj[(int64_t)u * n + a] = 0;\n", ""),
    "clique_last_pick_unchecked": (
        "    for (int32_t j = 0; j < c && ok; ++j) ok = adj[(int64_t)pick[j] * n + v] != 0;",
        "    for (int32_t j = 0; j + 1 < c && ok; ++j) ok = adj[(int64_t)pick[j] * n + v] != 0;"),
    "clique_ignores_live_mask": (
        "    if (colour[v] != c || (alive && !alive[v])) continue;", "    if (colour[v] != c) continue;"),
    "clique_descending_order": (
        "  for (int32_t v = 0; v < n; ++v) {\n    if (colour[v] != c",
        "  for (int32_t v = n - 1; v >= 0; --v) {\n    if (colour[v] != c"),
    "struction_ac_rule_one_endpoint": (
        "        else if (ys < 0) e = adj[(int64_t)xs * n + xt] && adj[(int64_t)xs * n + yt];",
        "        else if (ys < 0) e = adj[(int64_t)xs * n + xt];"),
    "struction_cc_rule_any_first_vertex": (
        "        else if (ys >= 0 && yt >= 0) e = xs == xt && adj[(int64_t)ys * n + yt];",
        "        else if (ys >= 0 && yt >= 0) e = adj[(int64_t)ys * n + yt];"),
    "struction_counts_pairs_reaching_into_a": (
        "      if (y != pivot && !adj[(int64_t)pivot * n + y] && adj[(int64_t)x * n + y]) ++nc;",
        "      if (y != pivot && adj[(int64_t)x * n + y]) ++nc;"),
    "dom_edge_single_sweep": ("    if (!any) break;\n    ++sweeps;\n  }\n  stats[0] = sweeps;\n  stats[1] = de;",
                              "    break;\n  }\n  stats[0] = sweeps;\n  stats[1] = de;"),
}


def run_mutant(name, path, old, new, tests, tmp_path):
    text = open(path).read()
    assert text.count(old) == 1, "mutation site not found: " + name
    srcs = []
    for f in (SRC, EXT):
        if f == path:
            m = tmp_path / os.path.basename(f)
            m.write_text(text.replace(old, new))
            srcs.append(str(m))
        else:
            srcs.append(f)
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-o", str(lib)] + srcs, check=True)
    env = dict(os.environ, KZ_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", tests)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    run_mutant(name, SRC, old, new, "test_oracle.py", tmp_path)


@pytest.mark.parametrize("name", sorted(EXT_MUTANTS))
def test_ext_pins_catch_planted_mistake(name, tmp_path):
    old, new = EXT_MUTANTS[name]
    run_mutant(name, EXT, old, new, "test_oracle_ext.py", tmp_path)
