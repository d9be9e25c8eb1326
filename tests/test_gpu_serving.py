"""Continuous-batching server: results alone == results in a mix (bitwise),
admission, per-request error isolation, many requests from several threads."""
import threading

import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


def _mixed_requests(seed=0, n=24):
    """Water boxes (OU frames) and molecule batches, dipole or polarizability."""
    rng = np.random.default_rng(seed)
    reqs = []
    mols = synth.molecules(200, seed=seed + 1)
    for k in range(n):
        kind = 1 + int(rng.integers(0, 2))
        nf = int(rng.integers(1, 6))
        if rng.random() < 0.5:
            n_side = int(rng.choice([4, 6]))
            pos, spc, cell = synth.water_box(n_side, 12.42 * n_side / 4, seed=seed * 100 + k, o_species=3, h_species=1)
            fr = synth.ou_trajectory(pos, spc, cell, nf, seed=k)
        else:
            start = int(rng.integers(0, 190))
            fr = mols.subset(range(start, start + nf))
        reqs.append((kind, fr))
    return reqs


@pytest.fixture(scope="module")
def models():
    return synth.model("molecule_dipole"), synth.model("molecule_polarizability")


def test_alone_equals_mix_and_matches_oracle(gpu_lib, models):
    reqs = _mixed_requests()
    ctx = gpu_lib.Context(0)
    gm = {1: gpu_lib.Model(ctx, models[0]), 2: gpu_lib.Model(ctx, models[1])}
    # alone: plain synchronous path, one request at a time
    alone = []
    for kind, fr in reqs:
        f = gpu_lib.tnep_eval_dipole if kind == 1 else gpu_lib.tnep_eval_polarizability
        alone.append(np.asarray(f(ctx, gm[kind], fr)).reshape(fr.n_frames, -1))
    srv = gpu_lib.Server(ctx, max_batch_atoms=4000, max_inflight=3)
    tickets = [srv.submit(gm[kind], fr) for kind, fr in reqs]
    mixed = []
    for t in tickets:
        st, lat, out = srv.wait(t)
        assert st == 0 and lat > 0
        mixed.append(out)
    stats = srv.stats()
    srv.stop()
    assert stats["requests"] == len(reqs)
    assert stats["launches"] < len(reqs)  # requests were batched together
    for (kind, fr), a, b in zip(reqs, alone, mixed):
        assert np.array_equal(a, b)
    for (kind, fr), b in list(zip(reqs, mixed))[:6]:
        ref, pa = oracle.eval_frames(models[kind - 1], fr, per_atom=True)
        assert frame_errors(b, ref.reshape(fr.n_frames, -1), pa, fr.offsets).max() <= TENSOR_TOL
    ctx.close()


def test_concurrent_submitters(gpu_lib, models):
    reqs = _mixed_requests(seed=5, n=40)
    ctx = gpu_lib.Context(0)
    gm = {1: gpu_lib.Model(ctx, models[0]), 2: gpu_lib.Model(ctx, models[1])}
    srv = gpu_lib.Server(ctx, max_batch_atoms=20000, max_inflight=2)
    results = [None] * len(reqs)

    def worker(idx):
        for i in idx:
            kind, fr = reqs[i]
            t = srv.submit(gm[kind], fr)
            results[i] = srv.wait(t)

    th = [threading.Thread(target=worker, args=(list(range(k, len(reqs), 4)),)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.stop()
    for (kind, fr), (st, lat, out) in zip(reqs, results):
        f = gpu_lib.tnep_eval_dipole if kind == 1 else gpu_lib.tnep_eval_polarizability
        assert st == 0
        assert np.array_equal(np.asarray(f(ctx, gm[kind], fr)).reshape(fr.n_frames, -1), out)
    ctx.close()


def test_admission_and_error_isolation(gpu_lib, models):
    ctx = gpu_lib.Context(0)
    gm = gpu_lib.Model(ctx, models[0])
    srv = gpu_lib.Server(ctx, budget_bytes=64 << 20, max_inflight=2)  # a 64 MiB pool
    big_pos, big_spc, big_cell = synth.water_box(16, 49.7, seed=3, o_species=3, h_species=1)
    big = synth.Frames(np.array([0, len(big_spc)], np.int64), big_pos, big_spc, big_cell[None], np.ones((1, 3), np.uint8))
    with pytest.raises(gpu_lib.TnepError) as e:
        srv.submit(gm, big)
    assert e.value.code == -6
    good = synth.molecules(3, seed=9)
    bad = synth.molecules(2, seed=10)
    bad.species[4] = 9
    t1, t2, t3 = srv.submit(gm, good.subset([0])), srv.submit(gm, bad), srv.submit(gm, good.subset([1, 2]))
    s1, _, o1 = srv.wait(t1)
    s2, _, _ = srv.wait(t2)
    s3, _, o3 = srv.wait(t3)
    srv.stop()
    assert (s1, s2, s3) == (0, -2, 0)
    ref = gpu_lib.tnep_eval_dipole(ctx, gm, good)
    assert np.array_equal(o1[0], ref[0]) and np.array_equal(o3, ref[1:])
    ctx.close()


def test_memory_gated_admission(gpu_lib, models):
    """The slots share one memory pool: requests whose largest frame needs more
    than half the pool (so two of them never fit at once) are all admitted,
    wait for memory while another slot holds it, and finish with the results of
    the plain path; the slots never hold more than the pool."""
    ctx = gpu_lib.Context(0)
    gm = {1: gpu_lib.Model(ctx, models[0]), 2: gpu_lib.Model(ctx, models[1])}
    reqs = []
    for k in range(6):
        pos, spc, cell = synth.water_box(8, 24.84, seed=70 + k, o_species=3, h_species=1)
        reqs.append((1 + k % 2, synth.ou_trajectory(pos, spc, cell, 3, seed=k)))
    alone = []
    for kind, fr in reqs:
        f = gpu_lib.tnep_eval_dipole if kind == 1 else gpu_lib.tnep_eval_polarizability
        alone.append(np.asarray(f(ctx, gm[kind], fr)).reshape(fr.n_frames, -1))
    # pool: about 1.6 times what one 1536-atom frame needs (learned capacities
    # of a first server run on the same inputs), so no two slots can hold a
    # frame's buffers at the same time
    probe = gpu_lib.Server(ctx, max_batch_atoms=1536, max_inflight=1)
    probe.wait(probe.submit(gm[1], reqs[0][1].subset([0])))
    one_frame = probe.stats()["peak_bytes"]
    probe.stop()
    pool = int(1.6 * one_frame)
    srv = gpu_lib.Server(ctx, budget_bytes=pool, max_batch_atoms=1536, max_inflight=3)
    tickets = [srv.submit(gm[kind], fr) for kind, fr in reqs]
    outs = []
    for t in tickets:
        st, _, out = srv.wait(t)
        assert st == 0
        outs.append(out)
    with pytest.raises(gpu_lib.TnepError) as e:  # a ticket is waited for once
        srv.wait(tickets[0])
    assert e.value.code == -1
    stats = srv.stats()
    pool_bytes, granted, waits = srv.memory()
    print("pool", pool_bytes, "one frame", one_frame, "peak granted", stats["peak_bytes"], "memory waits", waits,
          flush=True)
    srv.stop()
    assert pool_bytes == pool
    assert stats["peak_bytes"] <= pool
    assert 2 * one_frame > pool
    for a, b in zip(alone, outs):
        assert np.array_equal(a, b)
    ctx.close()


def test_stop_with_requests_in_flight(gpu_lib, models):
    """Stopping the server while a thread is blocked in a wait: stop drains the
    queue, the wait returns with its result, and only then is the server's
    memory freed."""
    import time

    ctx = gpu_lib.Context(0)
    gm = gpu_lib.Model(ctx, models[0])
    srv = gpu_lib.Server(ctx, max_batch_atoms=2000, max_inflight=1)
    mols = synth.molecules(400, seed=12)
    tickets = [srv.submit(gm, mols.subset(range(k, k + 20))) for k in range(0, 400, 20)]
    got = []

    def waiter():
        got.append(srv.wait(tickets[-1]))

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.3)  # the waiter is inside tnep_wait (or its request is done)
    srv.stop()
    th.join()
    assert len(got) == 1 and got[0][0] == 0
    ref = gpu_lib.tnep_eval_dipole(ctx, gm, mols.subset(range(380, 400)))
    assert np.array_equal(got[0][2], ref)
    ctx.close()
