"""Comparison helpers for GPU-vs-oracle parity.

Bars (fixed before any kernel was written):
  - integer streams, cursors, uniform entries, fp64 triangle trajectories and
    integer counts: bit-exact;
  - fp32 deviates: |gpu - ref| <= max(4 ulp32(M), 1e-6 M) where M is the
    result's condition-aware magnitude (the oracle supplies a bound per
    output that already includes M and, for chains, the propagated effect of
    earlier steps); results below 2^-126 in magnitude pass if the GPU value
    is also in [-2^-126, 2^-126] with the same sign or zero;
  - accept/reject decisions may differ only where the oracle's decision
    statistic lies within its tolerance of the threshold (margin <= 1); such
    a flip desynchronises the unit's pool cursors, so the unit is compared up
    to the flip and its flips are counted.
"""
from __future__ import annotations

import numpy as np

TINY = 2.0 ** -126


def ulp32(m):
    m = np.abs(np.asarray(m, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(m, TINY)))
    return np.where(m < TINY, 2.0 ** -149, 2.0 ** (e - 23))


def tol_of(m):
    m = np.abs(np.asarray(m, dtype=np.float64))
    return np.maximum(4.0 * ulp32(m), 1e-6 * m)


def within(gpu, ref, tol):
    """Elementwise pass mask under the fp32 bar."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    ok = np.abs(gpu - ref) <= tol
    tiny = np.abs(ref) < TINY
    tiny_ok = (np.abs(gpu) <= TINY) & ((np.sign(gpu) == np.sign(ref)) | (gpu == 0))
    both_nan = np.isnan(gpu) & np.isnan(ref)
    return ok | (tiny & tiny_ok) | both_nan


def compare_units(gpu, ref, tol, margin, units_of_slot, step_axis=True, margin_limit=1.0):
    """Compare [t][slot] arrays unit by unit, allowing permitted flips.

    Returns (n_bad, flipped_units): n_bad counts elements outside the bar
    that are not explained by a permitted decision flip; flipped_units is
    the set of units that diverged at a permitted flip (compared only up to
    that step)."""
    gpu = np.atleast_2d(gpu)
    ref = np.atleast_2d(ref)
    tol = np.atleast_2d(tol)
    margin = np.atleast_2d(margin)
    ok = within(gpu, ref, tol)
    live = ~(np.isnan(ref) & np.isnan(gpu))
    bad_total = 0
    flipped = set()
    for u in np.unique(units_of_slot):
        cols = np.where(units_of_slot == u)[0]
        okc = ok[:, cols] | ~live[:, cols]
        rows = np.where(~okc.all(axis=1))[0]
        if rows.size == 0:
            continue
        t0 = rows[0]
        m = margin[t0, cols]
        if np.nanmin(m) <= margin_limit:
            flipped.add(int(u))
        else:
            bad_total += int((~okc[t0:]).sum())
    return bad_total, flipped


def compare_rounds(gpu, ref, tol, margin, r0, r1, units_of_slot, margin_limit=1.0):
    """compare_units for [t][slot] traces whose slots draw in rounds (gamma
    chains): a unit's steps do not line up in time across slots, so the
    unit's first mismatch is the one that completed in the earliest round,
    rb.  A flip is made in a round of the flipped draw's life [r0, r1], and
    the flipped draw itself then mismatches, at r1 at the latest; so the
    mismatch is explained only by a draw with margin <= limit and
    r0 <= rb <= r1.  r0/r1 are the oracle's start and completion rounds per
    draw (-1 where no draw)."""
    gpu = np.atleast_2d(gpu)
    ref = np.atleast_2d(ref)
    ok = within(gpu, ref, np.atleast_2d(tol))
    drawn = np.atleast_2d(r1) >= 0
    r0 = np.atleast_2d(r0)
    r1 = np.atleast_2d(r1)
    margin = np.atleast_2d(margin)
    bad_total = 0
    flipped = set()
    for u in np.unique(units_of_slot):
        cols = np.where(units_of_slot == u)[0]
        badc = drawn[:, cols] & ~ok[:, cols]
        if not badc.any():
            continue
        rb = r1[:, cols][badc].min()
        cand = (drawn[:, cols] & (margin[:, cols] <= margin_limit) & (r0[:, cols] <= rb)
                & (rb <= r1[:, cols]))
        if cand.any():
            flipped.add(int(u))
        else:
            bad_total += int(badc.sum())
    return bad_total, flipped
