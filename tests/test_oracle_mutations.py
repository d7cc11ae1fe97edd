"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (a dropped
term, a wrong sign or index, a transposed operand, a wrong comparison),
loads the copy as a module and runs the pins of tests/test_oracle_pins.py
against it: at least one pin must fail.  Mistakes are planted on the CPU in
the oracle only.
"""
import os
import sys
import types

import numpy as np
import pytest

import tests.test_oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "glu_oracle.py")

MUTATIONS = [
    ("Eq.4 projects on the wrong endpoint",
     'g = np.einsum("nc,nc->n", Ip - Lj, e)', 'g = np.einsum("nc,nc->n", Ip - Li, e)'),
    ("Eq.4 without eps",
     'den = np.einsum("nc,nc->n", e, e) + eps\n                g =', 'den = np.einsum("nc,nc->n", e, e)\n                g ='),
    ("Eq.4 weight not clamped",
     "np.clip(g / np.where(den > 0, den, 1.0), 0.0, 1.0), 1.0)\n            rec",
     "g / np.where(den > 0, den, 1.0), 1.0)\n            rec"),
    ("interpolation weights swapped",
     "rec = al[:, None] * Li + (1.0 - al)[:, None] * Lj", "rec = al[:, None] * Lj + (1.0 - al)[:, None] * Li"),
    ("window one cell short",
     "    for dy in range(-r, r + 1):\n        for dx in range(-r, r + 1):\n            cy = qy + dy",
     "    for dy in range(-r, r + 1):\n        for dx in range(-r, r):\n            cy = qy + dy"),
    ("LR cell of a pixel shifted", "    qx = xs // s\n    out = []", "    qx = (xs + 1) // s\n    out = []"),
    ("strict improvement replaced by <=", "upd = vi & vj & (err < best)", "upd = vi & vj & (err <= best)"),
    ("Eq.5 weight on the wrong side",
     "om = np.where(den > 0, dist[idx] / np.where(den > 0, den, 1.0), 1.0)",
     "om = np.where(den > 0, da / np.where(den > 0, den, 1.0), 1.0)"),
    ("anchor is the farthest colour", "        upd = dd < da\n", "        upd = dd > da\n"),
    ("Eq.1 weights swapped in apply",
     "return al * Tf[np.asarray(a)] + (1.0 - al) * Tf[np.asarray(b)]",
     "return (1.0 - al) * Tf[np.asarray(a)] + al * Tf[np.asarray(b)]"),
    ("backward sends alpha G to b", "np.add.at(dT, b, (1.0 - al)[:, None] * Gf)", "np.add.at(dT, b, al[:, None] * Gf)"),
    ("backward dalpha sign", "Tf[a] - Tf[b])", "Tf[b] - Tf[a])"),
    ("rollback condition reversed", "keep = not (e1 > e0)", "keep = not (e1 < e0)"),
    ("literal reading re-searches the affected set", "        R = C\n",
     "        R = _affected_pixels(Q, h, w, H, W, s, k)\n"),
    ("trial error sums over one pixel", "e0 = float(st.E[R].sum())", "e0 = float(st.E[R[:1]].sum())"),
    ("replacement takes the smallest error", "pstar = int(members[int(np.argmax(Em))])",
     "pstar = int(members[int(np.argmin(Em))])"),
    ("4-connected components",
     "            for dy in (-1, 0, 1):\n                for dx in (-1, 0, 1):\n                    ny, nx",
     "            for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):\n                if True:\n                    ny, nx"),
    ("regular grid samples the block corner", "ys = np.minimum(np.arange(h) * s + s // 2, H - 1)",
     "ys = np.minimum(np.arange(h) * s, H - 1)"),
    ("GNU weight on the wrong endpoint", "alpha=np.ones(n), err=da", "alpha=np.zeros(n), err=da"),
    ("GNU takes the farthest colour", "        upd = dd < da\n        da = np.where(upd, dd, da)\n        a = np.where(upd, lin, a)",
     "        upd = dd > da\n        da = np.where(upd, dd, da)\n        a = np.where(upd, lin, a)"),
    ("gradient step uphill", "        Z = L - eta * D\n", "        Z = L + eta * D\n"),
    ("loss gradient without its factor 2", "    G = 2.0 * (I_hat - I)\n", "    G = (I_hat - I)\n"),
    ("snap keeps the last nearest pixel", "            p = int(members[int(np.argmin(dist))])  # first minimum",
     "            p = int(members[len(dist) - 1 - int(np.argmin(dist[::-1]))])"),
    ("snap block one column short", "            xs = np.arange(qx * s, min(W, qx * s + s))\n",
     "            xs = np.arange(qx * s, min(W, qx * s + s - 1))\n"),
    ("affected set limited to the component's cells",
     "cells[max(0, qy - r) : qy + r + 1, max(0, qx - r) : qx + r + 1] = True",
     "cells[qy, qx] = True"),
]


def _pins():
    return [
        lambda: P.test_segment_example_exhaustive("eps"),
        lambda: P.test_segment_example_fast("eps"),
        lambda: P.test_segment_orientation_swapped(),
        lambda: P.test_exhaustive_bruteforce_eps0(11, 7, 9, 3),
        lambda: P.test_fast_bruteforce(21),
        lambda: P.test_nearest_copy_gives_zero_error("exhaustive", 4, 16, 20),
        lambda: P.test_nearest_copy_gives_zero_error("fast", 3, 9, 12),
        lambda: P.test_alpha_range_and_gnu_bound("exhaustive"),
        lambda: P.test_window_one_is_guided_nearest(),
        lambda: P.test_affine_transfer_and_self_reconstruction(),
        lambda: P.test_downsample_point_and_box(),
        lambda: P.test_backward_finite_differences(),
        lambda: P.test_backward_adjoint_and_torch_autograd(),
        lambda: P.test_ccl8_matches_scipy(1),
        lambda: P.test_joint_recovers_missed_dot(),
        lambda: P.test_joint_invariants_on_voronoi(),
        lambda: P.test_joint_constructed_rollback(),
        lambda: P.test_joint_literal_reading_sums_the_component(),
        lambda: P.test_exact_ties_go_to_the_earliest_candidate(),
        lambda: P.test_joint_replacement_takes_the_largest_error(),
        lambda: P.test_self_upsampling_gradient_finite_differences(),
        lambda: P.test_snap_to_block_bruteforce(),
        lambda: P.test_gradient_joint_fixed_points(),
        lambda: P.test_gradient_joint_best_and_copies(),
        lambda: P.test_gnu_is_the_nearest_window_colour(),
    ]


def _load_mutant(old, new, monkeypatch):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: " + old[:60]
    mod = types.ModuleType("oracle_mutant")
    monkeypatch.setitem(sys.modules, "oracle_mutant", mod)
    exec(compile(src.replace(old, new, 1), "oracle_mutant", "exec"), mod.__dict__)
    return mod


def test_unmutated_oracle_passes_every_pin():
    for pin in _pins():
        pin()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, monkeypatch):
    mutant = _load_mutant(old, new, monkeypatch)
    monkeypatch.setattr(P, "O", mutant)
    failures = 0
    with np.errstate(all="ignore"):
        for pin in _pins():
            try:
                pin()
            except Exception:
                failures += 1
    assert failures >= 1, "no pin caught: " + name
