"""Choosing the number of probe modes by the rule of Section II (after Eq.
6): trial runs with one mode more each time, and the search ends at the
first run in which some mode carries less than 1% of the total intensity;
the count before it is kept.

The per-mode powers come from the library: best the eigen-powers of
`dm_orthogonalize_modes` (the eigenvalues of the modes' overlap matrix, which
a unitary mix of the modes leaves alone; the mix does not change the
intensity model of Eq. 1, so the plain powers of non-orthogonal modes,
`dm_mode_power`, depend on how a reconstruction happened to split the
power between them).  This module holds only the host-side bookkeeping of
the search.
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple


def mode_fractions(power: Sequence[float]) -> List[float]:
    """Share of each mode in the total intensity, power[k] / sum(power)."""
    total = float(sum(power))
    if total <= 0.0:
        return [0.0 for _ in power]
    return [float(p) / total for p in power]


def choose_mode_count(run: Callable[[int], Sequence[float]], max_modes: int,
                      threshold: float = 0.01,
                      start: int = 1) -> Tuple[int, List[Tuple[int, List[float]]]]:
    """run(M) reconstructs with M probe modes and returns the M mode powers
    (for example a DMContext's `orthogonalize_modes()` after some
    iterations).  M runs
    from `start` up to `max_modes`; the search stops at the first M whose
    smallest share is below `threshold` and returns the M before it (or
    `start`), with the shares of every trial run."""
    if start < 1 or max_modes < start:
        raise ValueError("need 1 <= start <= max_modes")
    chosen = start
    history: List[Tuple[int, List[float]]] = []
    for m in range(start, max_modes + 1):
        power = list(run(m))
        if len(power) != m:
            raise ValueError(f"run({m}) returned {len(power)} mode powers")
        shares = mode_fractions(power)
        history.append((m, shares))
        if min(shares) < threshold:
            break
        chosen = m
    return chosen, history
