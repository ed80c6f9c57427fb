"""Serving loop on the GPU: each request's results are bit-identical to the
same lookups filtered alone (stf_filter) whatever else is in the mix;
admission respects the memory budget and the resident limit; oversized
requests are rejected; pending requests can be cancelled; the open-loop
replay reports latency percentiles."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def textures():
    g1 = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=7)
    g2 = synth.fbm_grid((128, 64, 32), base_period=16.0, seed=8)
    t1 = stf.stf_create_sparse_grid3d(g1.dims, stf.STF_FMT_F16, g1.origins, g1.encoded("f16"))
    t2 = stf.stf_create_sparse_grid3d(g2.dims, stf.STF_FMT_F32, g2.origins, g2.values)
    tex = synth.texture2d(128, 96, 4, seed=9)
    t3 = stf.stf_create_texture2d(128, 96, 4, stf.STF_FMT_F16, [synth.encode(tex, "f16")])
    yield [(t1, g1.dims), (t2, g2.dims), (t3, None)]
    for t, _ in ((t1, 0), (t2, 0), (t3, 0)):
        t.destroy()


def _queries(tex_dims, n, rng):
    if tex_dims is None:
        return rng.random((n, 2), dtype=np.float32)
    return synth.uniform_box_queries(tex_dims, n, seed=int(rng.integers(1 << 30)), margin=2.0)


def _alone(dev, tex, q, filt, seed):
    qd = torch.from_numpy(q).to(dev)
    out, idx = stf.filter(tex, qd, filt, stf.STF_STOCHASTIC, seed, want_index=True)
    return out.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("on_device", [False, True])
def test_single_request_equals_plain_filter(dev, textures, on_device):
    srv = stf.stf_server_create(64 << 20, 16, 1000)
    rng = np.random.default_rng(1)
    for tex, dims in textures:
        q = _queries(dims, 5001, rng)
        ref, ridx = _alone(dev, tex, q, stf.STF_CUBIC_BSPLINE, 42)
        if on_device:
            qd = torch.from_numpy(q).to(dev)
            out = torch.empty(ref.shape, dtype=torch.float32, device=dev)
            idx = torch.empty(ridx.shape, dtype=torch.int32, device=dev)
            t = stf.stf_server_submit(srv, tex, qd, stf.STF_CUBIC_BSPLINE, 42, out, idx)
            stf.stf_server_wait(srv, t)
            got, gidx = out.cpu().numpy(), idx.cpu().numpy()
        else:
            got = np.empty_like(ref)
            gidx = np.empty_like(ridx)
            t = stf.stf_server_submit(srv, tex, q, stf.STF_CUBIC_BSPLINE, 42, got, gidx)
            stf.stf_server_wait(srv, t)
        assert stf.stf_server_poll(srv, t)
        assert np.array_equal(gidx, ridx)
        assert np.array_equal(np.nan_to_num(got, nan=-7), np.nan_to_num(ref, nan=-7))
        stf.stf_server_release(srv, t)
    srv.destroy()


def test_mixed_requests_are_bit_identical_to_alone(dev, textures):
    rng = np.random.default_rng(2)
    reqs = []
    for k in range(240):
        tex, dims = textures[int(rng.integers(3))]
        n = int(np.clip(np.exp(rng.normal(np.log(3000), 1.0)), 100, 40000))
        filt = stf.STF_CUBIC_BSPLINE if rng.random() < 0.5 else stf.STF_LINEAR
        reqs.append((tex, _queries(dims, n, rng), filt, int(rng.integers(1 << 62))))
    budget = 4 << 20     # far less than all requests together: admission queues them
    srv = stf.stf_server_create(budget, 32, 4096)
    outs = []
    tickets = []
    for tex, q, filt, seed in reqs:
        out = np.empty((q.shape[0], tex.channels), np.float32)
        idx = np.empty((q.shape[0], tex.dims), np.int32)
        tickets.append(stf.stf_server_submit(srv, tex, q, filt, seed, out, idx))
        outs.append((out, idx))
    for t in tickets:
        stf.stf_server_wait(srv, t)
    st = stf.stf_server_stats(srv)
    assert st["completed"] == len(reqs)
    assert st["peak_arena_bytes"] <= budget
    assert st["peak_resident"] <= 32
    assert st["rounds"] > 1
    for (tex, q, filt, seed), (out, idx) in zip(reqs, outs):
        ref, ridx = _alone(dev, tex, q, filt, seed)
        assert np.array_equal(idx, ridx)
        assert np.array_equal(np.nan_to_num(out, nan=-7), np.nan_to_num(ref, nan=-7))
    srv.destroy()


def test_oversized_request_is_rejected(dev, textures):
    srv = stf.stf_server_create(1 << 16, 4, 1024)
    tex, dims = textures[0]
    q = _queries(dims, 100000, np.random.default_rng(3))
    out = np.empty((100000, 1), np.float32)
    with pytest.raises(stf.STFError) as e:
        stf.stf_server_submit(srv, tex, q, stf.STF_LINEAR, 1, out)
    assert e.value.status == stf.STF_E_OOM
    srv.destroy()


def test_cancel_pending_request(dev, textures):
    srv = stf.stf_server_create(32 << 20, 1, 256)   # one resident request at a time, small chunks
    tex, dims = textures[0]
    rng = np.random.default_rng(4)
    big = _queries(dims, 400000, rng)
    small = _queries(dims, 1000, rng)
    out_big = np.empty((400000, 1), np.float32)
    out_small = np.empty((1000, 1), np.float32)
    t1 = stf.stf_server_submit(srv, tex, big, stf.STF_CUBIC_BSPLINE, 1, out_big)
    t2 = stf.stf_server_submit(srv, tex, small, stf.STF_CUBIC_BSPLINE, 2, out_small)
    stf.stf_server_cancel(srv, t2)
    with pytest.raises(stf.STFError) as e:
        stf.stf_server_wait(srv, t2)
    assert e.value.status == stf.STF_E_CANCELLED
    stf.stf_server_wait(srv, t1)
    ref, _ = _alone(dev, tex, big, stf.STF_CUBIC_BSPLINE, 1)
    assert np.array_equal(np.nan_to_num(out_big, nan=-7), np.nan_to_num(ref, nan=-7))
    st = stf.stf_server_stats(srv)
    assert st["cancelled"] == 1 and st["completed"] == 1
    srv.destroy()


def test_open_loop_replay_reports_latency(dev, textures):
    srv = stf.stf_server_create(256 << 20, 256, 1 << 16)
    tex, dims = textures[0]
    pool = torch.from_numpy(_queries(dims, 1 << 20, np.random.default_rng(5))).to(dev)
    outp = torch.empty((1 << 20, 1), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(6)
    reqs, t = [], 0.0
    for k in range(400):
        t += rng.exponential(1e-4)
        n = int(rng.integers(1000, 20000))
        off = int(rng.integers(0, (1 << 20) - n))
        reqs.append((tex, pool.data_ptr() + 12 * off, n, stf.STF_CUBIC_BSPLINE, k, outp.data_ptr() + 4 * off, None, t))
    stf.stf_server_replay(srv, reqs, stf.STF_SERVE_QUERIES_ON_DEVICE | stf.STF_SERVE_RESULTS_ON_DEVICE)
    st = stf.stf_server_stats(srv)
    print(st)
    assert st["completed"] == 400 and st["queries"] == sum(r[2] for r in reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    srv.destroy()


def test_replay_time_out_leaves_nothing_in_flight(dev, textures):
    # A replay that times out cancels what is still outstanding and returns
    # only once no request can write into its buffers any more: right after
    # the call nothing is pending or resident, and every request either
    # completed or was cancelled.
    srv = stf.stf_server_create(64 << 20, 4, 4096)
    tex, dims = textures[0]
    pool = torch.from_numpy(_queries(dims, 1 << 20, np.random.default_rng(7))).to(dev)
    outp = torch.empty((1 << 20, 1), dtype=torch.float32, device=dev)
    reqs = [(tex, pool.data_ptr(), 1 << 20, stf.STF_CUBIC_BSPLINE, k, outp.data_ptr(), None, 0.0) for k in range(16)]
    with pytest.raises(stf.STFError) as e:
        stf.stf_server_replay(srv, reqs, stf.STF_SERVE_QUERIES_ON_DEVICE | stf.STF_SERVE_RESULTS_ON_DEVICE,
                              timeout_s=0.0)
    assert e.value.status == stf.STF_E_BUSY
    st = stf.stf_server_stats(srv)
    assert st["pending"] == 0 and st["resident"] == 0
    assert st["completed"] + st["cancelled"] == 16 and st["cancelled"] > 0
    srv.destroy()


def test_device_results_in_place_and_flag_checks(dev, textures):
    # Device results are written in place: a request whose results alone
    # would overflow a small arena is admitted when they live on the device,
    # and its results equal stf_filter's.  Buffers flagged as device memory
    # that are not are rejected at submission.
    tex, dims = textures[2]   # 2D RGBA texture
    n = 100000
    q = _queries(dims, n, np.random.default_rng(8))
    ref, ridx = _alone(dev, tex, q, stf.STF_CUBIC_BSPLINE, 17)
    srv = stf.stf_server_create(1 << 16, 4, 8192)   # 64 KiB: far less than n x 16 B of results
    qd = torch.from_numpy(q).to(dev)
    out = torch.empty((n, tex.channels), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    t = stf.stf_server_submit(srv, tex, qd, stf.STF_CUBIC_BSPLINE, 17, out, idx)
    stf.stf_server_wait(srv, t)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert stf.stf_server_stats(srv)["peak_arena_bytes"] == 0
    L = stf._srv_lib()
    ticket = ctypes.c_uint64()
    host_out = np.empty((n, tex.channels), np.float32)
    host_q = np.ascontiguousarray(q)
    both = stf.STF_SERVE_QUERIES_ON_DEVICE | stf.STF_SERVE_RESULTS_ON_DEVICE
    # results flagged as device memory but on the host
    assert L.stf_server_submit(srv.handle, tex.handle, qd.data_ptr(), n, stf.STF_LINEAR, 1,
                               host_out.ctypes.data, None, both, ctypes.byref(ticket)) == stf.STF_E_INVALID
    # queries flagged as device memory but on the host
    assert L.stf_server_submit(srv.handle, tex.handle, host_q.ctypes.data, n, stf.STF_LINEAR, 1,
                               out.data_ptr(), None, both, ctypes.byref(ticket)) == stf.STF_E_INVALID
    # results far larger than the device allocation holding out (a small
    # tensor comes from a 2 MiB block of torch's allocator; the check sees
    # allocations, not tensors)
    big = 1 << 20
    qbig = torch.full((big, 2), 0.5, dtype=torch.float32, device=dev)
    small = torch.empty(1024, dtype=torch.float32, device=dev)
    assert L.stf_server_submit(srv.handle, tex.handle, qbig.data_ptr(), big, stf.STF_LINEAR, 1,
                               small.data_ptr(), None, both, ctypes.byref(ticket)) == stf.STF_E_INVALID
    srv.destroy()
