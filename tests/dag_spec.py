"""The multi-encoding DAG used by the GPU tests (proposed multi-encoding section).

Per resolution, five QPs; the median-QP job is the master of the other four (same
resolution: depths d-1..d+1, MV refinement r = 2); the masters chain across
resolutions (ratio 2: depths d..d+1, r = 4).
"""
DAG_QPS = (30, 22, 26, 34, 38)


def dag_rungs(sizes):
    """sizes: [(w, h, R)] from the lowest resolution up.  Returns one tuple per rung:
    (w, h, qp, R, ref rung index or -1, delta_lo, delta_hi, r)."""
    rungs = []
    for li, (w, h, R) in enumerate(sizes):
        base = 5 * li
        for k, qp in enumerate(DAG_QPS):
            if k == 0:
                ref = -1 if li == 0 else base - 5
                rungs.append((w, h, qp, R, ref, 0, 1, 4))
            else:
                rungs.append((w, h, qp, R, base, 1, 1, 2))
    return rungs
