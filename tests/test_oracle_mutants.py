"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of ``oracle/oracle.c`` (a
flipped comparison, a dropped condition, a wrong extremum), rebuilds that
copy, and runs the oracle pin tests against it in a subprocess: they must
fail.  CPU only; the real oracle is never modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    # H: '>= i' is the definition; '>' undercounts
    "hindex_strict": ("if (a[i - 1] >= i) h = (int32_t)i;",
                      "if (a[i - 1] > i) h = (int32_t)i;"),
    # H: sorting ascending instead of descending
    "hindex_sort_order": ("return (x < y) - (x > y);",
                          "return (x > y) - (x < y);"),
    # rho(S,R) is a minimum over the other r-cliques of S
    "rho_max": ("if (tau[ids->a[q * k + j]] < m) m",
                "if (tau[ids->a[q * k + j]] > m) m"),
    # peeling decrements only neighbours of strictly larger degree
    "peel_ge": ("if (ds[Rp] > ds[R]) {", "if (ds[Rp] >= ds[R]) {"),
    # peeling skips s-cliques that lost a processed r-clique
    "peel_no_skip": ("if (skip) continue;", "if (0) continue;"),
    # simple graph: no self-loops, no repeated pairs
    "keep_loops": ("if (a == b) continue;", "if (0) continue;"),
    "keep_repeats": (
        "if (i == 0 || key[i] != key[i - 1]) key[ne++] = key[i];",
        "key[ne++] = key[i];"),
    # degree levels: one decrement per removed s-clique
    "levels_double_count": ("if (gone_before || counted_by_other) continue;",
                            "if (gone_before) continue;"),
    # PartialAND: U on the listed r-cliques, not on the first |P| ids
    "update_set_index": ("update_body(&a->u, a->ids[i], wv);",
                         "update_body(&a->u, i, wv);"),
    # s-clique extension vertices must be pairwise adjacent
    "ext_not_clique": (
        "for (int j = 0; j < depth && ok; j++) ok = adjacent(g, c->ext[j], x);",
        ";"),
}

# Mistakes planted in oracle/__init__.py (the parts written in Python).
PY_MUTANTS = {
    # notifications reach neighbours whose value is >= the new one, not >
    "notify_strict": ("if h <= tau[Rp]:", "if h < tau[Rp]:"),
    # the listing's self-activation, which the worked example rules out
    "notify_self": ("self_activate: bool = False,", "self_activate: bool = True,"),
    # an iteration's work is the active set at its start
    "notify_live_set": ("for R in [R for R in visit if active[R]]:\n"
                        "                active[R] = False",
                        "for R in visit:\n"
                        "                if not active[R]:\n"
                        "                    continue\n"
                        "                active[R] = False"),
}

PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_invariants.py",
             "tests/test_oracle_partial.py"]


@pytest.mark.parametrize("name", sorted(MUTANTS) + sorted(PY_MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    fname = "oracle.c" if name in MUTANTS else "__init__.py"
    before, after = (MUTANTS if name in MUTANTS else PY_MUTANTS)[name]
    src = open(os.path.join(ROOT, "oracle", fname)).read()
    assert src.count(before) == 1, "mutation site moved"
    work = tmp_path / "repo"
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), work / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    (work / "oracle" / fname).write_text(src.replace(before, after))
    env = dict(os.environ, PYTHONPATH=str(work))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p",
                        "no:cacheprovider", *PIN_FILES], cwd=work, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, r.stdout[-2000:] + r.stderr[-2000:]
    assert "failed" in r.stdout
