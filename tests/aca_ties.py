"""Where a GPU ACA and the oracle's ACA of the same block part ways.

Algorithm 2 takes three kinds of decisions per step: the row pivot (largest
|residual column| over unused rows), the next column pivot (largest |v_r|
over unused columns) and the stopping test of Section 2.4.  The GPU path and
the oracle evaluate the same formulas in the same precision, but sum in
different orders, so their values differ in the last bits (more where the
residual has cancelled far below the block's entries).  Two runs of the
same algorithm can then only part ways at a decision that was a near tie:
two pivot candidates within a relative gap comparable to that rounding, or
a stopping ratio that sits on the threshold.

first_divergence() finds the first step at which the GPU's factor columns
leave the oracle's, and explain() reads the oracle's traced decisions at
that step.  A rank difference that is not explained by a near tie is a bug.
"""
import numpy as np


def first_divergence(Ug, Vg, Uo, Vo, rtol=1e-6):
    """First step s whose u_s or v_s differ (relative to the column's largest
    entry) beyond rtol, or min(rank_g, rank_o) when all common steps agree."""
    k = min(Ug.shape[1], Uo.shape[1])
    for s in range(k):
        for A, B in ((Ug[:, s], Uo[:, s]), (Vg[:, s], Vo[:, s])):
            scale = max(np.abs(B).max(), 1e-300)
            if np.abs(A - B).max() > rtol * scale:
                return s
    return k


def explain(trace, s, rank_g, rank_o, delta):
    """The oracle's near tie behind a divergence at step s: returns (kind,
    gap) with gap <= delta when the divergence is explained, else (kind of
    the closest decision, its gap).

    trace rows (one per accepted step of the oracle): row pivot, column,
    relative gap of the row pivot to the runner-up, stopping-test ratio
    |u||v| / (tol |S|) (stop at <= 1), relative gap of the next column pivot."""
    cands = []
    ro = trace.shape[0]
    if s < min(rank_g, rank_o):
        # the step's column or its row pivot differ
        if s < ro:
            cands.append(("row pivot", trace[s, 2]))
        if s >= 1:
            cands.append(("column pivot", trace[s - 1, 4]))
    else:
        # every common step agrees: one side stopped, the other went on
        last = min(rank_g, rank_o) - 1
        if 0 <= last < ro:
            cands.append(("stopping test", abs(trace[last, 3] - 1.0)))
    # a stop decided one step earlier or later on the other side also shows
    # as a near-threshold ratio just before s
    if 1 <= s <= ro:
        cands.append(("stopping test", abs(trace[s - 1, 3] - 1.0)))
    if not cands:
        return ("none", np.inf)
    kind, gap = min(cands, key=lambda c: c[1])
    return kind, gap
