"""Comparison rules between the GPU path and the FP64 oracle.

Scores: |Q_gpu - Q_64| <= max(rtol * |Q_64|, atol) with rtol = 1e-5, atol = 1e-7.

Indices: where several answers are correct (ties, near-ties inside the
float32 error), compare what is unique and check the rest is valid:
* every GPU top-N entry (t, s, q) is valid: the oracle's best Q of t and its
  Q at shift s both agree with q within the score tolerance;
* the GPU's ranked scores agree with the oracle's ranked scores;
* rank r's template must equal the oracle's wherever the oracle's score gap
  to both neighbouring ranks exceeds `margin` (1e-4 is the contract; tests
  also use a tight margin of twice the score tolerance);
* the angle must equal the oracle's wherever the oracle's angle margin
  (best Q minus the best Q at any other shift of that template) exceeds
  `margin`.
"""
from __future__ import annotations

import numpy as np

import oracle

RTOL = 1e-5
ATOL = 1e-7


def tol(q):
    return np.maximum(RTOL * np.abs(q), ATOL)


def scores_close(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) <= tol(ref)


class PatternRef:
    """FP64 oracle results for one pattern (full per-template table)."""

    def __init__(self, P64: np.ndarray, olib: "oracle.OracleLibrary", pnorm: float | None = None,
                 templates=None, best=None, arg=None):
        """best, arg (optional): the oracle's match_exact64 of the whole
        library for this pattern, computed elsewhere (oracle_best_pool)."""
        self.P = P64
        self.olib = olib
        self.pnorm = oracle.norm64(P64) if pnorm is None else pnorm
        lib = olib if templates is None else olib.subset(templates)
        self.ids = np.arange(olib.n_total) if templates is None else np.asarray(templates)
        if best is not None:
            assert templates is None
            self.Q = None
            self.best, self.arg = np.asarray(best), np.asarray(arg)
        else:
            self.Q = oracle.scores64(P64, lib, self.pnorm) if lib.n_total <= 6000 else None
            if self.Q is not None:
                self.best = self.Q.max(axis=1)
                self.arg = self.Q.argmax(axis=1)
            else:
                self.best, self.arg = oracle.match_exact64(P64, lib, self.pnorm)
        self.order = np.lexsort((self.ids, -self.best))
        self._pos = {int(t): i for i, t in enumerate(self.ids)}

    def q_at(self, t: int, s: int) -> float:
        i = self._pos[int(t)]
        if self.Q is not None:
            return float(self.Q[i, s])
        sub = self.olib.subset([int(t)])
        return float(oracle.scores64(self.P, sub, self.pnorm)[0, s])

    def angle_margin(self, t: int) -> float:
        i = self._pos[int(t)]
        if self.Q is not None:
            row = self.Q[i]
        else:
            row = oracle.scores64(self.P, self.olib.subset([int(t)]), self.pnorm)[0]
        srt = np.sort(row)
        return float(srt[-1] - srt[-2]) if len(srt) > 1 else np.inf


def check_topn(ref: PatternRef, gt, gs, gq, margin: float, tight: bool = True):
    """Assert the GPU top-N (gt, gs, gq) agrees with the oracle. Returns the
    number of ranks whose template index was checked exactly."""
    gt = np.asarray(gt)
    gs = np.asarray(gs)
    gq = np.asarray(gq, dtype=np.float64)
    N = len(gt)
    ot = ref.ids[ref.order[: N + 1]]
    oq = ref.best[ref.order[: N + 1]]
    # ranked scores
    ok = scores_close(gq, oq[:N])
    assert ok.all(), f"ranked scores differ: gpu {gq[~ok]} oracle {oq[:N][~ok]}"
    assert len(set(gt.tolist())) == N, "templates must be distinct"
    # validity of every entry
    for t, s, q in zip(gt, gs, gq):
        i = ref._pos[int(t)]
        assert scores_close(q, ref.best[i]), f"template {t}: gpu {q} oracle best {ref.best[i]}"
        assert scores_close(q, ref.q_at(t, s)), f"template {t} angle {s}: score at that angle differs"
    exact = 0
    for r in range(N):
        lo = oq[r] - oq[r + 1] if r + 1 < len(oq) else np.inf
        hi = oq[r - 1] - oq[r] if r > 0 else np.inf
        gap = min(lo, hi)
        need = margin if not tight else min(margin, 2.0 * float(tol(oq[r])) + 2.0 * float(tol(oq[min(r + 1, len(oq) - 1)])))
        if gap > need:
            assert int(gt[r]) == int(ot[r]), f"rank {r}: gpu template {gt[r]} oracle {ot[r]} gap {gap}"
            exact += 1
            am = ref.angle_margin(ot[r])
            i = ref._pos[int(ot[r])]
            if am > need:
                assert int(gs[r]) == int(ref.arg[i]), f"rank {r}: gpu angle {gs[r]} oracle {ref.arg[i]}"
    return exact


# ------------------------------------------------------------------ oracle pool
# The oracle's exact search over tens of thousands of templates takes half a
# minute or more per pattern on one core; full-size parity tests spread the
# sampled patterns over worker processes (spawned: no GPU state is shared).
# Each worker builds the workload's oracle library once.

_POOL = {}


def _pool_init(cid):
    import synth
    cfg = synth.WORKLOADS[cid]
    lib_np = synth.make_library(cfg)
    _POOL["cfg"] = cfg
    _POOL["olib"] = oracle.OracleLibrary.build(lib_np, synth.px_per_inv_A(cfg), cfg.R, cfg.n_theta)


def _pool_best(img):
    cfg, olib = _POOL["cfg"], _POOL["olib"]
    P = oracle.polar64(np.asarray(img, dtype=np.float64), cfg.R, cfg.n_theta)
    return oracle.match_exact64(P, olib, oracle.norm64(P))


def oracle_best_pool(cid, imgs, workers=16):
    """(best, arg) of oracle.match_exact64 for each image of workload cid."""
    import multiprocessing
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(max(1, min(workers, len(imgs))), initializer=_pool_init,
                  initargs=(cid,)) as pool:
        return pool.map(_pool_best, [np.asarray(im) for im in imgs], chunksize=1)
