"""Serving (continuous batching) through the csrec_server_* C-ABI.

Checks: every tile's result is bit-identical alone and in the mix (and equal
to the direct csrec_gomp call on the same tile); tiles of different band
counts share launches; admission waits for HBM budget and keeps arrival
order; a tile larger than the budget is refused with CSREC_E_BUDGET."""
import numpy as np
import pytest

import oracle
from gpu_common import GAP, GAP_ABS, note, np_of, rel_err_rows, require_gpu, to_dev
from paper_2401_14762_amd import workloads as W

pytestmark = pytest.mark.gpu
K, S, TOL = 20, 2, 1e-3


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _tiles():
    out = []
    for i, (side, N) in enumerate([(40, 100), (64, 200), (23, 224), (90, 200), (7, 100), (64, 224)]):
        M = W.m_for(N)
        _, a32, _, phi = W.serving_dictionary(N)
        F = W.mixing_spectra(side * side, N, 40.0, 500 + i)
        out.append((N, (F @ phi.T).astype(np.float32)))
    return out


def _dicts():
    return {N: W.serving_dictionary(N)[1] for N in (100, 200, 224)}


def _serve(cs, tiles, dicts, budget=1 << 30, batch=32768, chunk=4096):
    with cs.Server(K=K, S=S, res_tol=TOL, hbm_budget_bytes=budget, batch_pixels=batch, chunk_pixels=chunk) as srv:
        ids = {N: srv.add_dict(A) for N, A in dicts.items()}
        for tag, (N, Y) in enumerate(tiles):
            srv.submit(ids[N], Y, tag)
        srv.drain()
        res = {r["tag"]: r for r in srv.poll(1000)}
    return res


def test_alone_equals_mix_equals_direct(torch):
    import paper_2401_14762_amd as cs
    tiles, dicts = _tiles(), _dicts()
    note("serving: all tiles mixed")
    mix = _serve(cs, tiles, dicts)
    assert sorted(mix) == list(range(len(tiles)))
    for tag, (N, Y) in enumerate(tiles):
        note(f"serving: tile {tag} alone (N={N}, P={Y.shape[0]})")
        alone = _serve(cs, [(N, Y)], dicts)[0]
        assert mix[tag]["status"] == 0 and alone["status"] == 0
        assert np.array_equal(mix[tag]["X"], alone["X"]), tag
        assert np.array_equal(mix[tag]["support"], alone["support"]), tag
        X, Sup, st = cs.gomp(to_dev(torch, dicts[N]), to_dev(torch, Y), K=K, S=S, res_tol=TOL)
        torch.cuda.synchronize()
        assert np.array_equal(mix[tag]["X"], np_of(X)), tag
        assert np.array_equal(mix[tag]["support"], np_of(Sup)), tag
        assert np.array_equal(mix[tag]["iters"], np_of(st["iters"])), tag
    # oracle parity on one tile's pixels away from near-ties
    N, Y = tiles[1]
    ref = oracle.gomp(dicts[N], Y[:300], K=K, S=S, res_tol=TOL, diagnostics=True)
    clean = (ref["sel_gap"] >= GAP) & (ref["prune_gap"] >= GAP) & (ref["stop_margin"] >= 1e-3)
    clean &= (ref["sel_gap_abs"] >= GAP_ABS) & (ref["prune_gap_abs"] >= GAP_ABS)
    # K = 20 solves that end near the noise floor: about a quarter of the
    # pixels hold a decision within FP32 resolution of a tie
    assert clean.mean() > 0.7
    assert np.array_equal(mix[1]["support"][:300][clean], ref["support"][clean])
    assert rel_err_rows(mix[1]["X"][:300][clean], ref["X"][clean]).max() <= 1e-5


def test_budget_admission_and_order(torch):
    import paper_2401_14762_amd as cs
    tiles, dicts = _tiles(), _dicts()
    # a pool that holds about one large tile at a time: tiles wait for space
    big = max(Y.shape[0] * (Y.shape[1] + 224 + K + 4) * 4 for _, Y in tiles)
    note("serving: tight budget")
    res = _serve(cs, tiles, dicts, budget=int(big * 1.3) + 65536)
    admits = [res[t]["t_admit"] for t in range(len(tiles))]
    assert admits == sorted(admits)
    for t in range(len(tiles)):
        assert res[t]["t_submit"] <= res[t]["t_admit"] <= res[t]["t_done"]
    mix = _serve(cs, tiles, dicts)
    for t in range(len(tiles)):
        assert np.array_equal(res[t]["X"], mix[t]["X"])
    with cs.Server(K=K, S=S, res_tol=TOL, hbm_budget_bytes=1 << 20, batch_pixels=4096) as srv:
        d = srv.add_dict(dicts[200])
        with pytest.raises(cs.CsrecError) as ei:
            srv.submit(d, tiles[3][1], 0)
        assert ei.value.code == -6


def test_fp64_fallback_through_the_server(torch):
    """Nearly duplicated atoms with pivot_fallback: the grouped FP64 redo of the
    flagged pixels gives the same results as the direct csrec_gomp call, and
    meets the FP64 oracle on the pixels away from near-ties."""
    import paper_2401_14762_amd as cs
    rng = np.random.default_rng(11)
    M, N, P = 40, 100, 200
    A = rng.standard_normal((M, N)) / np.sqrt(M)
    A[:, 1] = A[:, 0] + 1e-5 * rng.standard_normal(M)
    A32 = A.astype(np.float32)
    X = np.zeros((P, N))
    X[:, 0] = 1.0
    X[:, 1] = 1.0
    X[np.arange(P), 5 + np.arange(P) % 50] = 0.5
    Y = (X @ A32.astype(np.float64).T).astype(np.float32)
    note("serving: fp64 fallback")
    with cs.Server(K=6, S=2, res_tol=1e-6, pivot_fallback=1e-6, hbm_budget_bytes=1 << 28, batch_pixels=4096,
                   chunk_pixels=64) as srv:
        did = srv.add_dict(A32)
        srv.submit(did, Y[:77], 0)
        srv.submit(did, Y[77:], 1)
        # a tile with its own FP32 error-estimate threshold (its own launch class)
        srv.submit(did, Y, 2, redo_tol=1e-9)
        srv.drain()
        res = {r["tag"]: r for r in srv.poll(10)}
    Xs = np.concatenate([res[0]["X"], res[1]["X"]])
    Ss = np.concatenate([res[0]["support"], res[1]["support"]])
    fl = np.concatenate([res[0]["flags"], res[1]["flags"]])
    assert res[0]["status"] == 0 and res[1]["status"] == 0
    Xd, Sd, std = cs.gomp(to_dev(torch, A32), to_dev(torch, Y), K=6, S=2, res_tol=1e-6, pivot_fallback=1e-6)
    torch.cuda.synchronize()
    assert np.array_equal(Xs, np_of(Xd)) and np.array_equal(Ss, np_of(Sd))
    fb = (fl & oracle.STOP_FALLBACK) != 0
    assert fb.any() and np.array_equal(fl, np_of(std["flags"]).view(np.uint32))
    ref = oracle.gomp(A32, Y, K=6, S=2, res_tol=1e-6, diagnostics=True)
    ok = fb & (ref["sel_gap"] >= GAP) & (ref["prune_gap"] >= GAP)
    assert ok.any()
    assert rel_err_rows(Xs[ok], ref["X"][ok]).max() < 1e-5
    # redo_tol per tile: equal to the direct call with it, no fewer FP64 redos
    X9, S9, st9 = cs.gomp(to_dev(torch, A32), to_dev(torch, Y), K=6, S=2, res_tol=1e-6, pivot_fallback=1e-6,
                          redo_tol=1e-9)
    torch.cuda.synchronize()
    assert res[2]["status"] == 0
    assert np.array_equal(res[2]["X"], np_of(X9)) and np.array_equal(res[2]["support"], np_of(S9))
    fl9 = res[2]["flags"]
    assert np.array_equal(fl9, np_of(st9["flags"]).view(np.uint32))
    assert ((fl9 & oracle.STOP_FALLBACK) != 0).sum() >= fb.sum()


def test_per_tile_parameters_and_tags(torch):
    """Tiles with their own res_tol / max_iter / prune share the server with
    tiles on its defaults; each equals the direct csrec_gomp call with its own
    parameters.  A tag still in use is refused; a released one is reusable."""
    import paper_2401_14762_amd as cs
    tiles, dicts = _tiles(), _dicts()
    own = {1: dict(res_tol=1e-2), 3: dict(max_iter=12, prune="final"), 4: dict(res_tol=0.0, max_iter=5),
           5: dict(prec="bf16"), 2: dict(prec="f16")}
    note("serving: per-tile parameters")
    with cs.Server(K=K, S=S, res_tol=TOL, hbm_budget_bytes=1 << 30, batch_pixels=32768, chunk_pixels=4096) as srv:
        ids = {N: srv.add_dict(A) for N, A in dicts.items()}
        for tag, (N, Y) in enumerate(tiles):
            srv.submit(ids[N], Y, tag, **own.get(tag, {}))
        with pytest.raises(cs.CsrecError) as ei:
            srv.submit(ids[tiles[0][0]], tiles[0][1], 0)
        assert ei.value.code == -1
        with pytest.raises(cs.CsrecError) as ei:
            srv.submit(ids[100], tiles[0][1], 99, K=K + 1)
        assert ei.value.code == -5
        srv.drain()
        res = {r["tag"]: r for r in srv.poll(1000)}
        # polled and released by poll(): tag 0 may be used again
        srv.submit(ids[tiles[0][0]], tiles[0][1], 0)
        srv.drain()
        again = srv.poll(10)
        st = srv.stats()
    assert len(again) == 1 and np.array_equal(again[0]["X"], res[0]["X"])
    for tag, (N, Y) in enumerate(tiles):
        kw = dict(K=K, S=S, res_tol=TOL)
        kw.update(own.get(tag, {}))
        X, Sup, sd = cs.gomp(to_dev(torch, dicts[N]), to_dev(torch, Y), **kw)
        torch.cuda.synchronize()
        assert res[tag]["status"] == 0
        assert np.array_equal(res[tag]["X"], np_of(X)), tag
        assert np.array_equal(res[tag]["support"], np_of(Sup)), tag
        assert np.array_equal(res[tag]["iters"], np_of(sd["iters"])), tag
    assert st["tiles_submitted"] == len(tiles) + 1 and st["tiles_finished"] == len(tiles) + 1
    assert st["pixels_launched"] == sum(Y.shape[0] for _, Y in tiles) + tiles[0][1].shape[0]
    assert 0 < st["busy_s"] <= st["elapsed_s"] and st["mean_pixels_in_flight"] > 0


def test_results_held_with_a_small_host_pool(torch):
    """A caller that polls but releases nothing while the pinned staging pool
    (64 MiB, its minimum, with a 64 MiB device budget) is far smaller than the
    results: every tile still finishes (results beyond the pool go to
    pageable memory), and each equals the run with a large pool."""
    import paper_2401_14762_amd as cs
    dicts = _dicts()
    _, a32, _, phi = W.serving_dictionary(224)
    tiles = []
    for i in range(10):
        F = W.mixing_spectra(128 * 128, 224, 40.0, 900 + i)
        tiles.append((224, (F @ phi.T).astype(np.float32)))
    note("serving: results held, 64 MiB pinned pool, 10 tiles of 16384 pixels at N=224")
    got = {}
    with cs.Server(K=K, S=S, res_tol=TOL, hbm_budget_bytes=64 << 20, batch_pixels=32768,
                   chunk_pixels=8192) as srv:
        d = srv.add_dict(dicts[224])
        for tag, (_, Y) in enumerate(tiles):
            srv.submit(d, Y, tag)
        held = []
        while len(got) < len(tiles):
            for r in srv.poll_held(16):
                got[r["tag"]] = r
                held.append(r["tag"])
        srv.drain()
        st = srv.stats()
        for tag in held:
            srv.release(tag)
    assert st["host_out_pageable"] > 0
    ref = _serve(cs, tiles, dicts, budget=1 << 30)
    for tag in range(len(tiles)):
        assert got[tag]["status"] == 0
        assert np.array_equal(got[tag]["X"], ref[tag]["X"]), tag
