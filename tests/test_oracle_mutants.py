"""The pins must catch plausible mistakes in the oracle.

Each mutant is a copy of the C oracle with one deliberate mistake (a dropped
term, a flipped comparison, a wrong index, swapped operands...), compiled to
a private shared object in a temporary directory.  A small battery drawn from
the pin tests (brute force on tie-heavy inputs, the 1-D closed form, the
worked example and special cases) is run against it in a child process; every
mutant must fail at least one check.  Nothing here touches the real oracle
library or the GPU.
"""
import json
import os
import subprocess
import sys
import textwrap

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sbm_body(src):
    start = src.index("static int sbm(")
    end = src.index("/* Public entry points")
    return start, end


MUTANTS = {
    # half-open filter on the other axes becomes closed
    "closed_other_axes": ("all", "return before(rd, a_low, b_high) && before(rd, b_low, a_high);",
                          "return a_low <= b_high && b_low <= a_high;"),
    # ties sort lower-before-upper
    "lower_before_upper": ("all", "    return type == TYPE_UPPER ? 0 : 1;",
                           "    return type == TYPE_LOWER ? 0 : 1;"),
    # ties by coordinate only
    "coordinate_only_order": ("all", "if (x->rank != y->rank) return x->rank < y->rank ? -1 : 1;",
                              "return 0;"),
    # empty regions kept in the sweep
    "keep_empties": ("all", "if (is_empty(rd, ulo, uhi, i, d)) continue;", ""),
    # other axes never tested
    "no_axis_filter": ("all", "for (int k = 1; k < d; ++k)", "for (int k = 1; k < 1; ++k)"),
    # wrong axis range in the filter (0..d-2 instead of 1..d-1)
    "filter_axis_off_by_one": ("all", "for (int k = 1; k < d; ++k)", "for (int k = 0; k < d - 1; ++k)"),
    # pairs at update uppers dropped
    "drop_update_upper_emission": ("sbm", "report(&s, e->id, sb);", "(void)sb;"),
    # ids swapped when reporting at subscription uppers
    "swapped_report_operands": ("sbm", "report(&s, u, e->id);", "report(&s, e->id, u);"),
    # the sweep uses axis d-1 for the update upper endpoints
    "sweep_wrong_axis": ("all", "T[t++] = (Endpoint){(double)uhi[i * d], TYPE_UPPER, ru, KIND_UPD, i};",
                         "T[t++] = (Endpoint){(double)uhi[i * d + (d - 1)], TYPE_UPPER, ru, KIND_UPD, i};"),
    # the lower endpoint of subscriptions is taken from the upper array
    "lower_from_upper_array": ("all", "T[t++] = (Endpoint){(double)slo[j * d], TYPE_LOWER, rl, KIND_SUB, j};",
                               "T[t++] = (Endpoint){(double)shi[j * d], TYPE_LOWER, rl, KIND_SUB, j};"),
    # per-update histogram indexed by the subscription id
    "histogram_by_sub": ("all", "if (s->per_update) s->per_update[upd] += 1;",
                         "if (s->per_update) s->per_update[sub % 1] += 1;"),
    # validation forgets lo > hi
    "no_order_validation": ("all", "if (l > h) return OR_E_INVAL;", ""),
    # pairs not sorted at the end
    "unsorted_pairs": ("all", "qsort(s->pairs, (size_t)s->count, 2 * sizeof(int32_t), cmp_pair);", ""),
    # closed reading: ties sort upper-before-lower
    "closed_upper_first": ("all", "if (rd->closed) return type == TYPE_LOWER ? 0 : 1;",
                           "if (rd->closed) return type == TYPE_UPPER ? 0 : 1;"),
    # closed reading: points (lo == hi) dropped as if empty
    "closed_drops_points": ("all", "if (rd->closed) return 0;", ""),
    # closed reading: strict comparisons
    "closed_strict": ("all", "return rd->closed ? a <= b : a < b;", "return a < b;"),
}


BATTERY = textwrap.dedent(r"""
    import json, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_1703_06680_amd import workloads as W
    o = O.Oracle(LIB)
    fails = []
    def check(name, cond):
        if not cond:
            fails.append(name)
    # worked example of Sec. 3
    g = json.load(open(GOLDEN))
    a = [np.asarray(g[k], dtype=np.float32) for k in ("upd_lo", "upd_hi", "sub_lo", "sub_hi")]
    try:
        check("example", o.sbm(*a)[2].tolist() == g["expected_pairs"])
    except Exception:
        fails.append("example-raised")
    # plain definition on tie-heavy and float inputs
    for d in (1, 2, 3):
        for seed in range(25):
            for inst in (W.tie_heavy(19, 19, d, seed=seed), W.random_float_boxes(19, 19, d, seed=seed)):
                a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
                hit = O.bruteforce_numpy(*a)
                try:
                    k, per, pairs = o.sbm(*a)
                except Exception:
                    fails.append("raised"); continue
                check("count", k == int(hit.sum()))
                check("pairs", np.array_equal(pairs, O.pairs_from_matrix(hit)))
                check("per_update", np.array_equal(per, hit.sum(axis=1).astype(np.int32)))
    # closed intervals: the plain definition with <=, and its 1-D closed form
    for d in (1, 2, 3):
        for seed in range(15):
            inst = W.tie_heavy(19, 19, d, seed=seed)
            a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
            hit = O.bruteforce_numpy(*a, closed=True)
            try:
                k, per, pairs = o.sbm(*a, closed=True)
            except Exception:
                fails.append("closed-raised"); continue
            check("closed-count", k == int(hit.sum()))
            check("closed-pairs", np.array_equal(pairs, O.pairs_from_matrix(hit)))
            if d == 1:
                check("closed-form", np.array_equal(per.astype(np.int64),
                                                    O.closed_form_1d(*a, closed=True)))
    # closed form on one axis
    inst = W.uniform_instance(3000, 3000, 1, 1.0, seed=1)
    a = (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)
    try:
        k, per, _ = o.sbm(*a, pairs=False)
        check("closed_form", np.array_equal(per.astype(np.int64), O.closed_form_1d(*a)))
    except Exception:
        fails.append("closed_form-raised")
    # validation
    try:
        o.sbm(np.array([[2.0]], np.float32), np.array([[1.0]], np.float32),
              np.array([[0.0]], np.float32), np.array([[1.0]], np.float32))
        fails.append("validation")
    except O.OracleError as e:
        check("validation-code", e.code == O.OR_E_INVAL)
    print(json.dumps(sorted(set(fails))))
""")


def _run_battery(lib, tmp):
    # the script lives in a directory of its own so that nothing next to it
    # can shadow a standard module
    os.makedirs(os.path.join(tmp, "battery"), exist_ok=True)
    script = os.path.join(tmp, "battery", "pin_battery.py")
    with open(script, "w") as f:
        f.write(f"ROOT = {ROOT!r}\nLIB = {lib!r}\nGOLDEN = "
                f"{os.path.join(ROOT, 'tests', 'golden', 'ddm_example_fig.json')!r}\n")
        f.write(BATTERY)
    r = subprocess.run([sys.executable, script], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        # a mutant may corrupt memory and die; the unmutated copy must not
        return ["crashed: " + r.stderr[-300:]]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_unmutated_copy_passes_the_battery(tmp_path):
    src = open(O.SOURCE).read()
    path = tmp_path / "oracle_unmutated.c"
    path.write_text(src)
    lib = O.build(str(path), str(tmp_path / "liboracle_unmutated.so"))
    assert _run_battery(lib, str(tmp_path)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    scope, old, new = MUTANTS[name]
    src = open(O.SOURCE).read()
    if scope == "sbm":
        a, b = _sbm_body(src)
        body = src[a:b]
        assert old in body, name
        src = src[:a] + body.replace(old, new) + src[b:]
    else:
        assert old in src, name
        src = src.replace(old, new)
    path = tmp_path / f"oracle_mutant_{name}.c"
    path.write_text(src)
    lib = O.build(str(path), str(tmp_path / f"liboracle_mutant_{name}.so"))
    fails = _run_battery(lib, str(tmp_path))
    assert fails, f"mutant {name} passed every pin"
