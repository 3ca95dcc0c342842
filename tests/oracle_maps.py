"""Whole disparity maps from the CPU oracle for large frames, one oracle call
per view in parallel threads (the oracle itself is single-threaded C; ctypes
releases the interpreter lock during each call).  Test infrastructure only."""
from concurrent.futures import ThreadPoolExecutor


def _view(orc, base, match, D, base_is_right, P1, P2):
    S = orc.aggregate(orc.cost(orc.census(base), orc.census(match), D, base_is_right), P1, P2)
    return orc.wta(S)


def maps(orc, pairs, D, P1=10, P2=120, tol=1, threads=4, left_only=False):
    """pairs: list of (left, right) uint8 images.  Returns, per pair, a dict with
    the left WTA, the unmasked left sub-pixel map, and (unless left_only) the
    LR-checked disparity map and its mask."""
    jobs = []
    for L, R in pairs:
        jobs.append((L, R, False))
        if not left_only:
            jobs.append((R, L, True))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda j: _view(orc, j[0], j[1], D, j[2], P1, P2), jobs))
    out = []
    step = 1 if left_only else 2
    for i in range(len(pairs)):
        wl, dsub = res[step * i]
        m = {"wta_left": wl, "dsub": dsub}
        if not left_only:
            wr, _ = res[step * i + 1]
            valid, disp = orc.lr_check(wl, wr, dsub, tol)
            m.update(wta_right=wr, valid=valid, disp=disp)
        out.append(m)
    return out
