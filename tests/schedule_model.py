"""A host model of the work decomposition the device prologue builds for one
epoch (test infrastructure): which work units exist, in which ticket group
each one sits, and which other units each one waits for.

It is written from the decomposition's rules, not from the kernels' code:

- batch k of epoch e holds the positions [k b, min(n, (k+1) b)) of the
  epoch's partition; vertex v belongs to batch pos(v) // b;
- a row of degree at most `chunk` is one WHOLE unit: its CSR list, then the
  batch's s shared negatives, then the step;
- a longer row is split: its list is divided into a LATE part (entries of the
  W batches just before the row's own) and an EARLY part (all other entries);
  the early part is cut into EARLY units of `chunk` entries whose partial sums
  are combined; the LATE unit takes the late part and the negatives, waits for
  the combined early sum and takes the step;
- a unit of batch k that reads a row of an earlier batch waits until the unit
  that finishes that row (its whole or late unit) has published it;
- ticket order: per batch j, a first part (the whole units of batch j, then
  the early units of batch j + W, or of batches 0..W for j = 0) padded to a
  multiple of the lane-group count S, then a second part (the late units of
  batch j) padded the same way; ticket t is processed in group t // S.

The model is used to check the property the device schedules rely on for
deadlock freedom: every unit waits only for units in strictly lower groups.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Unit:
    kind: str        # "whole", "early" or "late"
    u: int           # vertex whose row the unit works on
    k: int           # batch of u
    entries: np.ndarray  # vertex ids read (neighbours, then negatives for whole/late units)
    ticket: int = -1


def default_chunk(n: int) -> int:
    return 64 if n >= 750_000 else 32


def default_window(n: int) -> int:
    return 28 if n >= 750_000 else 24


def lane_groups(d: int) -> int:
    """Rows processed together by one wave (S = 64 / G): G lanes per row,
    two elements per lane, at least 8 and at most 64 lanes."""
    lanes = max(1, (d + 1) // 2)
    g = 8
    while g < lanes and g < 64:
        g *= 2
    return 64 // g


def build_epoch(rowptr, colidx, perm, negs, b: int, chunk: int, window: int, slots: int):
    """Units of one epoch with their tickets.  perm: position -> vertex;
    negs: [nb, s] shared negatives.  Returns (units, batch_of_vertex, finisher)
    where finisher[v] is the index of the unit that publishes v's row."""
    n = len(perm)
    nb = (n + b - 1) // b
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    bat = pos // b
    deg = np.diff(rowptr)
    whole = [[] for _ in range(nb)]
    early = [[] for _ in range(nb)]
    late = [[] for _ in range(nb)]
    units: list[Unit] = []
    finisher = np.full(n, -1, dtype=np.int64)
    early_of = {}
    for p in range(n):
        u = int(perm[p])
        k = p // b
        lst = colidx[rowptr[u]:rowptr[u + 1]]
        neg = negs[k] if negs.size else np.zeros(0, dtype=np.int64)
        if deg[u] <= chunk:
            units.append(Unit("whole", u, k, np.concatenate([lst, neg])))
            whole[k].append(len(units) - 1)
            finisher[u] = len(units) - 1
        else:
            kb = bat[lst]
            is_late = (kb < k) & (kb >= k - window)
            ep, lp = lst[~is_late], lst[is_late]
            mine = []
            for c in range(0, len(ep), chunk):
                units.append(Unit("early", u, k, ep[c:c + chunk]))
                early[k].append(len(units) - 1)
                mine.append(len(units) - 1)
            early_of[u] = mine
            units.append(Unit("late", u, k, np.concatenate([lp, neg])))
            late[k].append(len(units) - 1)
            finisher[u] = len(units) - 1
    t = 0
    for j in range(nb):
        first = list(whole[j])
        if j == 0:
            for kk in range(0, min(window, nb - 1) + 1):
                first += early[kk]
        elif j + window < nb:
            first += early[j + window]
        for i in first:
            units[i].ticket = t
            t += 1
        t = (t + slots - 1) // slots * slots
        for i in late[j]:
            units[i].ticket = t
            t += 1
        t = (t + slots - 1) // slots * slots
    return units, bat, finisher, early_of


def check_waits_lower(units, bat, finisher, early_of, slots: int) -> dict:
    """For every unit: the groups of the units it waits for are strictly lower
    than its own.  Returns counts and the worst margin (own group minus the
    highest awaited group; positive everywhere means the property holds)."""
    worst = None
    waits = 0
    for w in units:
        assert w.ticket >= 0
        g = w.ticket // slots
        deps = []
        if w.entries.size:
            older = w.entries[bat[w.entries] < w.k]
            deps += [int(finisher[v]) for v in older]
        if w.kind == "late":
            deps += early_of.get(w.u, [])
        for dep in deps:
            waits += 1
            m = g - units[dep].ticket // slots
            worst = m if worst is None or m < worst else worst
    return {"units": len(units), "waits": waits, "worst_margin": worst}
