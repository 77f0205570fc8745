"""Serving path: batched ragged maps and the continuous-batching server (GPU).

* srp_map_nyquist_batched gives, for every array, bit-identical maps whether
  the array is launched alone or mixed with others, equal to srp_map_nyquist
  (FP32) within 1e-5 and to the FP64 oracle within 1e-5; with BF16/FP16
  samples (matrix cores, up to 16 frames per array) within 1e-2 of the oracle,
  again bit-identical alone and mixed.
* The server admits arrays by memory (an array that does not fit waits and is
  admitted when another closes), fails bad requests alone, and returns for
  every frame the same peak as the frame processed alone (bit-identical in
  FP32; in BF16 within the BF16 tolerance, since the kernel a frame runs on
  depends on how many frames of its array share its batch).
* A fault injected into one batch's launch fails that batch alone; frames
  done after their deadline are counted, and with shedding a frame whose
  deadline passed before its batch is failed without running.
"""
import time

import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests import refpath as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2012_09499_amd as srp  # noqa: E402
from paper_2012_09499_amd import serving as SV  # noqa: E402


def _arrays(frames=(1, 3, 2, 8), ff_frames=2):
    # mixed microphone counts, windows and grid sizes; one far-field array
    specs = [dict(M=4, J_shape=(17, 9, 5), L=1024, seed=21),
             dict(M=8, J_shape=(11, 13, 7), L=1024, seed=22),
             dict(M=16, J_shape=(9, 7, 5), L=1024, seed=23),
             dict(M=5, J_shape=(31, 3, 3), L=1024, seed=24)]
    out = [WL.make_custom(h=0.12, F=F, **sp) for sp, F in zip(specs, frames)]
    ff = WL.make_far_field(F=ff_frames, L=1024, step_deg=6.0)
    out.append(ff)
    return out


LOWP_FRAMES = dict(frames=(1, 3, 16, 2), ff_frames=11)


def _geom(wl):
    return srp.Geometry(wl.mic_xyz, wl.candidates(), fs=wl.fs, L=wl.L, c=wl.c, n_aux=wl.n_aux,
                        field=wl.field)


def _batched(entries, dtype="fp32"):
    """entries: list of (geom, frames tensor). Returns per-entry (map, peaks)."""
    xis, items, outs = [], [], []
    off = 0
    for g, fr in entries:
        psi = srp.cross_spectra(g, fr)
        xis.append(srp.gcc_samples(g, psi, dtype=dtype).reshape(-1))
    arena = torch.cat(xis)
    for (g, fr), x in zip(entries, xis):
        F = fr.shape[0]
        m = torch.empty((F, g.J), dtype=torch.float32, device="cuda")
        pk = torch.empty((F, 2), dtype=torch.int64, device="cuda")
        items.append((g, off, F, m, pk))
        outs.append((m, pk))
        off += x.numel()
    ws = torch.empty(srp.batched_workspace_bytes(len(items)), dtype=torch.uint8, device="cuda")
    srp.map_nyquist_batched(items, arena, ws, dtype=dtype)
    torch.cuda.synchronize()
    return outs


def test_batched_alone_equals_mixed_and_single_kernel_and_oracle():
    wls = _arrays()
    geoms = [_geom(w) for w in wls]
    frames = [torch.from_numpy(w.frames).cuda() for w in wls]
    mixed = _batched(list(zip(geoms, frames)))
    for i, (w, g, fr) in enumerate(zip(wls, geoms, frames)):
        alone = _batched([(g, fr)])[0]
        assert torch.equal(alone[0], mixed[i][0]) and torch.equal(alone[1], mixed[i][1])
        m_single, _ = srp.map_nyquist(g, srp.gcc_samples(g, srp.cross_spectra(g, fr)))
        got = mixed[i][0].cpu().numpy().astype(np.float64)
        assert O.rel_error(got, m_single.cpu().numpy()).max() <= 1e-5
        ref = R.oracle_nyquist(w, R.oracle_xi(w, R.oracle_psi(w)), w.candidates())
        assert O.rel_error(got, ref).max() <= 1e-5
        idx = srp.decode_peaks(mixed[i][1])[0]
        np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
        R.check_argmax(idx, ref, 1e-5, label=f"serving-batched/{i}/fp32")


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_batched_lowp_alone_equals_mixed_and_oracle(dtype):
    """BF16/FP16 samples on matrix cores: 1 to 16 frames per array, ragged
    candidate tails; bit-identical alone and mixed, within 1e-2 of the oracle."""
    wls = _arrays(**LOWP_FRAMES)
    geoms = [_geom(w) for w in wls]
    frames = [torch.from_numpy(w.frames).cuda() for w in wls]
    mixed = _batched(list(zip(geoms, frames)), dtype)
    for i, (w, g, fr) in enumerate(zip(wls, geoms, frames)):
        alone = _batched([(g, fr)], dtype)[0]
        assert torch.equal(alone[0], mixed[i][0]) and torch.equal(alone[1], mixed[i][1])
        got = mixed[i][0].cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all()
        ref = R.oracle_nyquist(w, R.oracle_xi(w, R.oracle_psi(w)), w.candidates())
        err = O.rel_error(got, ref)
        assert err.max() <= 1e-2, (dtype, i, err.max())
        idx = srp.decode_peaks(mixed[i][1])[0]
        np.testing.assert_array_equal(idx, np.argmax(got, axis=1))
        R.check_argmax(idx, ref, 1e-2, label=f"serving-batched/{i}/{dtype}")


def test_batched_argument_checks():
    w = _arrays()[0]
    g = _geom(w)
    fr = torch.from_numpy(np.concatenate([w.frames] * 17)).cuda()
    psi = srp.cross_spectra(g, fr)
    ws = torch.empty(srp.batched_workspace_bytes(1), dtype=torch.uint8, device="cuda")
    pk = torch.empty((17, 2), dtype=torch.int64, device="cuda")
    x32 = srp.gcc_samples(g, psi).reshape(-1)
    x16 = srp.gcc_samples(g, psi, dtype="bf16").reshape(-1)
    with pytest.raises(srp.SrpError, match="F must be in"):      # 9 frames in FP32
        srp.map_nyquist_batched([(g, 0, 9, None, pk[:9])], x32, ws)
    with pytest.raises(srp.SrpError, match="F must be in"):      # 17 frames in BF16
        srp.map_nyquist_batched([(g, 0, 17, None, pk)], x16, ws, dtype="bf16")
    with pytest.raises(srp.SrpError, match="multiple of 8"):
        srp.map_nyquist_batched([(g, 4, 1, None, pk[:1])], x16, ws, dtype="bf16")
    with pytest.raises(srp.SrpError, match="16-byte aligned"):
        srp.map_nyquist_batched([(g, 0, 1, None, pk[:1])], x16[1:], ws, dtype="bf16")
    with pytest.raises(TypeError):
        srp.map_nyquist_batched([(g, 0, 1, None, pk[:1])], x32, ws, dtype="bf16")
    # an item's F x S samples must lie inside the arena
    with pytest.raises(srp.SrpError, match="past the end"):      # arena of one frame
        srp.map_nyquist_batched([(g, 0, 2, None, pk[:2])], x32[:g.S], ws)
    with pytest.raises(srp.SrpError, match="past the end"):      # offset near the end
        srp.map_nyquist_batched([(g, 16 * g.S + 8, 1, None, pk[:1])], x16, ws, dtype="bf16")
    with pytest.raises(srp.SrpError, match="past the end"):      # offset past the end
        srp.map_nyquist_batched([(g, 18 * g.S, 1, None, pk[:1])], x32, ws)
    # the checks happen before anything runs: a valid call still works afterwards
    srp.map_nyquist_batched([(g, 0, 16, None, pk[:16])], x16, ws, dtype="bf16")
    torch.cuda.synchronize()
    idx = srp.decode_peaks(pk[:16])[0]
    assert ((idx >= 0) & (idx < g.J)).all()


def _serve(server, wls, ids, order):
    reqs = []
    for k, (ai, fi) in enumerate(order):
        reqs.append(server.submit(ids[ai], wls[ai].frames[fi]))
        if k % 3 == 0:
            server.pump()
    server.drain()
    return reqs


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_server_mixed_equals_alone(dtype):
    wls = _arrays() if dtype == "fp32" else _arrays(**LOWP_FRAMES)
    ids = list(range(len(wls)))
    srv = SV.SrpServer(dtype=dtype)
    for i, w in zip(ids, wls):
        assert srv.open_array(i, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c,
                              n_aux=w.n_aux, field=w.field)
    rng = np.random.default_rng(1)
    order = [(a, f) for a in range(len(wls)) for f in range(wls[a].F)]
    order = [order[j] for j in rng.permutation(len(order))]
    mixed = _serve(srv, wls, ids, order)
    assert all(r.status == "done" for r in mixed)
    assert srv.batches >= 1
    for r, (ai, fi) in zip(mixed, order):
        solo = SV.SrpServer(dtype=dtype)
        w = wls[ai]
        solo.open_array(0, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c, n_aux=w.n_aux,
                        field=w.field)
        s = solo.submit(0, w.frames[fi])
        solo.drain()
        assert s.status == "done"
        if dtype == "fp32":
            # one kernel, one summation order per candidate: bit-identical
            assert s.peak_index == r.peak_index and s.peak_value == r.peak_value
        else:
            # BF16: a frame runs on the vector or the matrix-core kernel depending
            # on how many frames of its array share the batch, so the two results
            # agree to the BF16 tolerance (and pick the same peak unless two peaks
            # are that close)
            assert abs(s.peak_value - r.peak_value) <= 1e-2 * abs(s.peak_value)
            if s.peak_index != r.peak_index:
                ref = R.oracle_nyquist(w, R.oracle_xi(w, R.oracle_psi(w)),
                                       w.candidates_at([s.peak_index, r.peak_index]))[fi]
                assert abs(ref[0] - ref[1]) <= 2e-2 * abs(ref[0])


def test_server_admission_by_memory_and_failures():
    wls = _arrays()[:3]
    needs = []
    for w in wls:
        N_p, off, Ssz = srp.pair_layout(w.mic_xyz, w.c, w.fs / 2, w.n_aux)
        needs.append(SV.footprint(w.J, w.M, w.L // 2 + 1, w.L, Ssz, w.P, int(N_p.max()) + w.n_aux))
    # array 2 fits alone, but not next to arrays 0 and 1
    srv = SV.SrpServer(memory_budget=needs[0] + needs[1] + needs[2] - 1)
    assert srv.open_array(0, wls[0].mic_xyz, wls[0].candidates(), fs=wls[0].fs, L=wls[0].L)
    assert srv.open_array(1, wls[1].mic_xyz, wls[1].candidates(), fs=wls[1].fs, L=wls[1].L)
    assert not srv.open_array(2, wls[2].mic_xyz, wls[2].candidates(), fs=wls[2].fs, L=wls[2].L)
    assert srv.admitted == [0, 1]
    bad = [srv.submit(2, wls[2].frames[0]),                      # not admitted yet
           srv.submit(0, wls[0].frames[0][:, :10]),              # wrong shape
           srv.submit(1, np.full_like(wls[1].frames[0], np.nan))]  # non-finite
    good = [srv.submit(0, wls[0].frames[0]), srv.submit(1, wls[1].frames[1])]
    srv.drain()
    assert all(r.status == "failed" and r.error for r in bad)
    assert all(r.status == "done" for r in good)
    srv.close_array(0)
    assert srv.admitted == [1, 2]
    r = srv.submit(2, wls[2].frames[1])
    srv.drain()
    assert r.status == "done"


def test_server_poisson_stream_runs_and_reports():
    """A short Poisson stream over mixed arrays: every frame completes, stats are sane."""
    wls = _arrays()
    srv = SV.SrpServer()
    for i, w in enumerate(wls):
        srv.open_array(i, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c, n_aux=w.n_aux,
                       field=w.field)
    rng = np.random.default_rng(3)
    t_end, rate = 0.5, 200.0
    arrivals = []
    for i, w in enumerate(wls):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= t_end:
                break
            arrivals.append((t, i))
    arrivals.sort()
    t0 = time.perf_counter()
    k = 0
    while k < len(arrivals) or any(s.event is not None for s in srv.slots):
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k][0] <= now:
            t, i = arrivals[k]
            srv.submit(i, wls[i].frames[k % wls[i].F], t_arrival=t0 + t)
            k += 1
        srv.pump()
    srv.drain()
    st = srv.stats(time.perf_counter() - t0)
    assert st["frames_done"] == len(arrivals) and st["frames_failed"] == 0
    assert st["latency_ms_p99"] >= st["latency_ms_p50"] > 0


def test_server_injected_batch_failure_fails_only_that_batch():
    """A fault injected into the second batch's launch fails that batch's frames
    alone: the batches before and after it complete, and a frame served after
    the failure gives the same peak as before it (FP32: bit-identical)."""
    wls = _arrays()[:2]
    batches = []

    def hook(reqs):
        batches.append(len(reqs))
        if len(batches) == 2:
            raise RuntimeError("injected launch failure")

    srv = SV.SrpServer(fault_hook=hook)
    for i, w in enumerate(wls):
        assert srv.open_array(i, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c,
                              n_aux=w.n_aux, field=w.field)

    def wave():
        reqs = [srv.submit(i, w.frames[0]) for i, w in enumerate(wls)]
        srv.drain()
        return reqs

    first, second, third = wave(), wave(), wave()
    assert len(batches) == 3
    assert all(r.status == "done" for r in first + third)
    assert all(r.status == "failed" and "injected" in r.error for r in second)
    for a, b in zip(first, third):
        assert (a.peak_index, a.peak_value) == (b.peak_index, b.peak_value)
    st = srv.stats(1.0)
    assert st["failed_batches"] == 1 and st["frames_failed"] == len(second)
    assert st["frames_done"] == len(first) + len(third)


def test_server_deadline_accounting_and_shedding():
    """Frames done after their deadline are counted; with shedding, a frame whose
    deadline has passed before its batch is assembled fails without running."""
    w = _arrays()[0]
    srv = SV.SrpServer(deadline_ms=1e-3)  # 1 us: every frame misses it
    assert srv.open_array(0, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c, n_aux=w.n_aux)
    reqs = [srv.submit(0, w.frames[0]) for _ in range(3)]
    srv.drain()
    assert all(r.status == "done" and r.missed for r in reqs)
    st = srv.stats(1.0)
    assert st["deadline_misses"] == 3 and st["deadline_miss_rate"] == 1.0
    shed = SV.SrpServer(deadline_ms=50.0, shed_expired=True)
    assert shed.open_array(0, w.mic_xyz, w.candidates(), fs=w.fs, L=w.L, c=w.c, n_aux=w.n_aux)
    late = shed.submit(0, w.frames[0], t_arrival=time.perf_counter() - 1.0)
    fresh = shed.submit(0, w.frames[0])
    shed.drain()
    assert late.status == "failed" and late.error == "deadline passed"
    assert fresh.status == "done" and not fresh.missed
    assert shed.stats(1.0)["shed_expired"] == 1
