"""Pins of the oracle's treatment of the rows below the diagonal (P_s).

Section 2.3 moves the rows below the diagonal of an eliminated cluster to
the neighbour clusters, each row to the cluster holding most of its squared
norm (the maximum-norm heuristic of Section 2.2); Section 4.2 counts the
sparsification of those rows in the reassign phase, and the per-level
runtime figure skips sparsification on the first two leaf-side levels.
The oracle reads this as: a column-pivoted QR of the extra-row block E
keeps the leading rows of Q^T E; on sparsified levels its rank follows the
rule |R_ii| >= eps |R_11| of Section 4, on the skipped levels it stops only
at the numerical rank (|R_ii| <= 1000 u ||E||_F).

The checks here restate that rule in closed form, independently of the code
that applies it:

* every kept pivot satisfies the rule (|R_ii| >= eps_l |R_11|, above the
  floor), so a missing truncation fails;
* what is dropped is bounded by the rule: ||E||_F^2 - ||kept rows||_F^2
  <= (n - r) max(eps_l |R_11|, floor)^2 (every dropped column is no larger
  than the rejected pivot), so a truncation that should not happen fails;
* the owner of a row is the neighbour with the largest squared mass, the
  lowest cluster id on ties (a hand-worked fixture);
* a rank-deficient block stops at its exact rank.
"""
import numpy as np
import pytest

from oracle import dense, spaqr
from synth import grid_ls

U = np.finfo(np.float64).eps / 2


def _run_logged(grid, depth, eps, skip, seed=0, extra=None):
    n = int(np.prod(grid))
    p = grid_ls(grid, n if extra is None else extra, seed)
    an = spaqr.analyze(p, depth)
    log = []
    f = spaqr.factorize(an, eps, skip, log=log)
    return an, f, log


def _reassign_checks(log, eps, depth, skip):
    """(rule_ok, bound_ok, n_truncated_by_eps) over the reassign records."""
    rule_ok, bound_ok, ntrunc = True, True, 0
    for rec in log:
        if rec["kind"] != "reassign":
            continue
        sparsified = 2 <= rec["level"] <= depth - skip
        eps_l = eps if sparsified else 0.0
        r, n, m = rec["rank"], rec["n"], rec["m"]
        rows, perm = rec["rows"], rec["perm"]
        floor = 1000.0 * U * np.sqrt(rec["normf2"])
        if r == 0:
            kept2, r11 = 0.0, 0.0
        else:
            diag = np.abs(rows[np.arange(r), perm])
            r11 = diag[0]
            if (diag < eps_l * r11).any() or (diag <= floor).any():
                rule_ok = False
            kept2 = float(np.sum(rows * rows))
        dropped2 = rec["normf2"] - kept2
        lim = max(eps_l * r11, floor)
        if dropped2 > (n - r) * lim * lim * (1 + 1e-6) + 1e-12 * rec["normf2"]:
            bound_ok = False
        if sparsified and r < min(m, n) and dropped2 > (n - r) * floor * floor * 1e4:
            ntrunc += 1
    return rule_ok, bound_ok, ntrunc


CASES = [((32, 32), 4, 1e-2, 1), ((24, 20), 4, 1e-1, 1), ((8, 8, 8), 4, 1e-2, 1)]


@pytest.mark.parametrize("grid,depth,eps,skip", CASES)
def test_reassign_rank_rule_closed_form(grid, depth, eps, skip):
    an, f, log = _run_logged(grid, depth, eps, skip)
    rule_ok, bound_ok, ntrunc = _reassign_checks(log, eps, depth, skip)
    assert rule_ok and bound_ok
    # not vacuous: the rule truncated some block on a sparsified level, and
    # the skipped leaf level has blocks of its own
    assert ntrunc > 0
    assert any(rec["kind"] == "reassign" and rec["level"] > depth - skip for rec in log)


def test_skipped_levels_keep_numerical_rank():
    # On the leaf level (not sparsified) the kept rows span E up to rounding:
    # the dropped part is at the numerical-rank floor, far below eps.
    an, f, log = _run_logged((32, 32), 4, 1e-1, 1)
    leaf = [rec for rec in log if rec["kind"] == "reassign" and rec["level"] == 4]
    assert leaf
    for rec in leaf:
        dropped2 = rec["normf2"] - float(np.sum(rec["rows"] ** 2))
        assert dropped2 <= 1e-12 * rec["normf2"]


def test_planted_missing_truncation_is_caught(monkeypatch):
    orig = spaqr._State.pivoted

    def bad(self, C, kind, eps=None):
        return orig(self, C, kind, 0.0 if kind == "reassign" else eps)
    monkeypatch.setattr(spaqr._State, "pivoted", bad)
    an, f, log = _run_logged((32, 32), 4, 1e-2, 1)
    rule_ok, bound_ok, _ = _reassign_checks(log, 1e-2, 4, 1)
    assert not rule_ok


def test_planted_truncation_on_skipped_levels_is_caught(monkeypatch):
    orig = spaqr._State.pivoted

    def bad(self, C, kind, eps=None):
        return orig(self, C, kind, self.eps if kind == "reassign" else eps)
    monkeypatch.setattr(spaqr._State, "pivoted", bad)
    an, f, log = _run_logged((32, 32), 4, 1e-1, 1)
    rule_ok, bound_ok, _ = _reassign_checks(log, 1e-1, 4, 1)
    assert not bound_ok


# ---- owner of a reassigned row ----------------------------------------------

def _owner_fixture():
    """Two neighbour clusters: c1 holds columns 0-1, c2 columns 2-3.

    row 0: [3, 0 | 1, 1]  mass 9 vs 2    -> c1
    row 1: [1, 1 | 0, 2]  mass 2 vs 4    -> c2
    row 2: [1, 0 | 0, 1]  mass 1 vs 1    -> tie, lowest id: c1
    row 3: [0, 0 | 0, 0]  mass 0 vs 0    -> tie, lowest id: c1
    row 4: [0, 1 | 2, 0]  mass 1 vs 4    -> c2
    """
    rows = np.array([[3.0, 0, 1, 1], [1, 1, 0, 2], [1, 0, 0, 1], [0, 0, 0, 0], [0, 1, 2, 0]])
    c1 = spaqr.Cluster(key=(3, 0), sep=None, gran=0, lo=(0, 0, 0), hi=(0, 0, 0))
    c2 = spaqr.Cluster(key=(3, 7), sep=None, gran=0, lo=(0, 0, 0), hi=(0, 0, 0))
    st = spaqr._State.__new__(spaqr._State)
    st.reassign_rows(rows, np.arange(4), [c1, c2], [(0, 2), (2, 4)], None)
    got1 = c1.groups[0].data if c1.groups else np.zeros((0, 4))
    got2 = c2.groups[0].data if c2.groups else np.zeros((0, 4))
    return (len(c1.groups) <= 1 and len(c2.groups) <= 1 and np.array_equal(got1, rows[[0, 2, 3]])
            and np.array_equal(got2, rows[[1, 4]]))


def test_owner_is_max_mass_lowest_id_on_ties():
    assert _owner_fixture()


def test_planted_min_mass_owner_is_caught(monkeypatch):
    def bad(self, rows, slots, clus, col_ranges, source):
        out = {}
        for i in range(rows.shape[0]):
            best, bestv = None, np.inf
            for c, (a, b) in zip(clus, col_ranges):
                v = float(np.dot(rows[i, a:b], rows[i, a:b]))
                if v < bestv:
                    best, bestv = c, v
            out.setdefault(best, []).append(i)
        for c in sorted(out, key=lambda c: c.key):
            c.groups.append(spaqr.Group(owner=c, data=rows[out[c]].copy(), slots=slots.copy(), clus=set(clus)))
    monkeypatch.setattr(spaqr._State, "reassign_rows", bad)
    assert not _owner_fixture()


def test_planted_highest_id_tie_break_is_caught(monkeypatch):
    def bad(self, rows, slots, clus, col_ranges, source):
        out = {}
        for i in range(rows.shape[0]):
            best, bestv = None, -1.0
            for c, (a, b) in zip(clus, col_ranges):
                v = float(np.dot(rows[i, a:b], rows[i, a:b]))
                if v >= bestv:
                    best, bestv = c, v
            out.setdefault(best, []).append(i)
        for c in sorted(out, key=lambda c: c.key):
            c.groups.append(spaqr.Group(owner=c, data=rows[out[c]].copy(), slots=slots.copy(), clus=set(clus)))
    monkeypatch.setattr(spaqr._State, "reassign_rows", bad)
    assert not _owner_fixture()


# ---- numerical-rank floor ------------------------------------------------------

def test_floor_stops_rank_one_block():
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal(6), rng.standard_normal(5)
    E = np.outer(u, v)
    r, rows, perm, V, tau = dense.pivoted_qr(E, 0.0)
    assert r == 1
    # the kept row carries all of E: |R_11| = ||u|| ||v||_inf at the largest |v_j|
    assert perm[0] == int(np.argmax(np.abs(v)))
    assert abs(abs(rows[0, perm[0]]) - np.linalg.norm(u) * np.abs(v).max()) <= 1e-13 * np.linalg.norm(E)
    assert abs(np.sum(rows ** 2) - np.sum(E ** 2)) <= 1e-13 * np.sum(E ** 2)


def test_floor_stops_dependent_columns():
    rng = np.random.default_rng(12)
    B = rng.standard_normal((7, 2))
    E = np.column_stack([B[:, 0], B[:, 1], B[:, 0] - 2 * B[:, 1], 3 * B[:, 1]])
    r, rows, perm, V, tau = dense.pivoted_qr(E, 0.0)
    assert r == 2
    assert abs(np.sum(rows ** 2) - np.sum(E ** 2)) <= 1e-13 * np.sum(E ** 2)


def test_floor_is_relative_to_frobenius_norm():
    # a column 1e-11 below the others is kept at eps = 0, one 1e-15 below is not
    rng = np.random.default_rng(13)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 3)))
    for scale, rank in ((1e-11, 3), (1e-15, 2)):
        E = np.column_stack([Q[:, 0], Q[:, 1], scale * Q[:, 2]])
        r, *_ = dense.pivoted_qr(E, 0.0)
        assert r == rank, (scale, r)
