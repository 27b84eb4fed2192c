"""Serving on the GPU: continuous batching of scan rows over three resident
libraries; each row's result is bit-identical alone and in the mix, and
agrees with the FP64 oracle. Marked gpu."""
import numpy as np
import pytest

import oracle
import synth
from parity import PatternRef, check_topn

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    import paper_2111_07347_amd as tm
    from paper_2111_07347_amd.serve import GpuExecutor, Server
    cfg0 = synth.serving_config(0)
    grid = tm.PolarGrid(R=cfg0.R, n_theta=cfg0.n_theta, cx=cfg0.cx, cy=cfg0.cy)
    px = synth.px_per_inv_A(cfg0)
    libs_np = {i: synth.make_library(synth.serving_config(i)) for i in range(3)}
    libs = {i: tm.Library(l["kx"], l["ky"], l["intensity"], l["offsets"], px, grid)
            for i, l in libs_np.items()}
    n_rows = 6
    lib_ids, _ = synth.serving_schedule(n_rows)
    lib_ids = np.array([0, 1, 2, 2, 1, 0])     # every library, repeated
    # 64 patterns per row keep the oracle checks short
    rows_np = [synth.serving_row(r, int(lib_ids[r]), libs_np[int(lib_ids[r])])[:64]
               for r in range(n_rows)]
    rows = [torch.from_numpy(r.view(np.int16)).pin_memory() for r in rows_np]
    return tm, GpuExecutor, Server, grid, px, libs_np, libs, lib_ids, rows_np, rows


def _serve(setup, order, slots, max_rows, burst=True, keep=0.0):
    tm, GpuExecutor, Server, grid, px, libs_np, libs, lib_ids, rows_np, rows = setup
    from paper_2111_07347_amd.serve import run_stream
    ex = GpuExecutor(libs, grid, N=5, slots=slots, prefilter_keep=keep)
    srv = Server(ex, budget_bytes=8 << 30, slots=slots, max_batch_rows=max_rows)
    res = run_stream(srv, [rows[i] for i in order], [lib_ids[i] for i in order],
                     np.zeros(len(order)) if burst else np.arange(len(order)) * 0.01)
    assert all(r.error is None for r in res)
    return {order[r.req_id]: r for r in res}


def test_alone_equals_mix(setup):
    n = len(setup[7])
    _say("serving: each row alone")
    alone = {}
    for i in range(n):
        alone.update(_serve(setup, [i], slots=1, max_rows=1))
    _say("serving: all rows mixed, 3 slots, batches of up to 3 rows")
    mix = _serve(setup, list(range(n)), slots=3, max_rows=3)
    assert max(r.batch_rows for r in mix.values()) > 1      # batching happened
    _say("serving: reversed order, paced arrivals")
    mix2 = _serve(setup, list(reversed(range(n))), slots=2, max_rows=2, burst=False)
    for i in range(n):
        for other in (mix[i], mix2[i]):
            assert np.array_equal(alone[i].top_template, other.top_template)
            assert np.array_equal(alone[i].top_angle, other.top_angle)
            assert np.array_equal(alone[i].top_score, other.top_score)


def test_serving_matches_oracle(setup):
    tm, GpuExecutor, Server, grid, px, libs_np, libs, lib_ids, rows_np, rows = setup
    res = _serve(setup, list(range(len(rows))), slots=3, max_rows=2)
    for i in (0, 1, 2):           # one row per library
        lib = libs_np[int(lib_ids[i])]
        cfg = synth.serving_config(int(lib_ids[i]))
        olib = oracle.OracleLibrary.build(lib, px, cfg.R, cfg.n_theta)
        for b in (0, 31):
            _say("serving oracle check row", i, "library", int(lib_ids[i]), "pattern", b)
            P = oracle.polar64(rows_np[i][b].astype(np.float64), cfg.R, cfg.n_theta)
            ref = PatternRef(P, olib)
            r = res[i]
            check_topn(ref, r.top_template[b], r.top_angle[b], r.top_score[b], margin=1e-4,
                       tight=True)


def test_fourier_route_library_serves_the_plain_results(setup):
    """A library served through the Fourier route with certified rescoring
    returns exactly the plain path's top-N, alone and in the mix."""
    tm, GpuExecutor, Server, grid, px, libs_np, libs, lib_ids, rows_np, rows = setup
    from paper_2111_07347_amd.serve import run_stream
    l2 = libs_np[2]
    libs_f = dict(libs)
    libs_f[2] = tm.Library(l2["kx"], l2["ky"], l2["intensity"], l2["offsets"], px, grid, fft=True)
    n = len(lib_ids)
    _say("serving: library 2 through the Fourier route, mixed, 3 slots")
    ex = GpuExecutor(libs_f, grid, N=5, slots=3, fourier={2})
    srv = Server(ex, budget_bytes=16 << 30, slots=3, max_batch_rows=3)
    res = run_stream(srv, rows, list(lib_ids), np.zeros(n))
    assert all(r.error is None for r in res)
    plain = _serve(setup, list(range(n)), slots=3, max_rows=3)
    for r in res:
        p = plain[r.req_id]
        assert np.array_equal(r.top_template, p.top_template), (r.req_id, lib_ids[r.req_id])
        assert np.array_equal(r.top_angle, p.top_angle), (r.req_id, lib_ids[r.req_id])
        assert np.array_equal(r.top_score, p.top_score), (r.req_id, lib_ids[r.req_id])


def test_window_bound_libraries_serve_the_plain_results(setup):
    """Every library served through the window-bound exact search returns
    exactly the plain path's top-N, in the mix."""
    tm, GpuExecutor, Server, grid, px, libs_np, libs, lib_ids, rows_np, rows = setup
    from paper_2111_07347_amd.serve import run_stream
    n = len(lib_ids)
    _say("serving: all libraries through the window-bound search, mixed, 3 slots")
    ex = GpuExecutor(libs, grid, N=5, slots=3, bound=set(libs))
    srv = Server(ex, budget_bytes=16 << 30, slots=3, max_batch_rows=3)
    res = run_stream(srv, rows, list(lib_ids), np.zeros(n))
    assert all(r.error is None for r in res)
    plain = _serve(setup, list(range(n)), slots=3, max_rows=3)
    for r in res:
        p = plain[r.req_id]
        assert np.array_equal(r.top_template, p.top_template), (r.req_id, lib_ids[r.req_id])
        assert np.array_equal(r.top_angle, p.top_angle), (r.req_id, lib_ids[r.req_id])
        assert np.array_equal(r.top_score, p.top_score), (r.req_id, lib_ids[r.req_id])
