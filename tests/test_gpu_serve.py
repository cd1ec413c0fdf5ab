"""Render server (sph_hoa_server_*): resident indices, request queue, continuous batching.

Every image served in a mix of concurrent requests must equal, bit for bit, the image
sph_hoa_render gives for the same camera alone, whichever batch and lane carried it; admission by
the memory budget decides how requests share batches and how many batches run at once; requests
arriving while a batch runs start on a free lane; errors surface at submission or at the wait.
"""
import threading

import pytest

import synth
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - needs a GPU
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2401_02896_amd as L  # noqa: E402

VMAX, STEP = 4.0e4, 1.4 / 256


def _cams():
    base = synth.tiny_camera()
    persp = {"eye": [0.5, 0.5, -1.0], "look_at": [0.5, 0.5, 0.5], "up": [0.0, 1.0, 0.0], "fov_y_deg": 40.0,
             "ortho": 0, "ortho_half_extent": 0.0, "width": 40, "height": 32, "t_min": 0.5, "t_max": 2.5}
    cams = []
    for i in range(12):
        if i % 3 == 0:
            cams.append(dict(base, width=8 + 4 * i, height=16))
        elif i % 3 == 1:
            cams.append(dict(persp, width=24 + i, height=20, fov_y_deg=20.0 + 2 * i))
        else:
            cams.append(dict(base, eye=[-0.2, 0.5, 0.5], look_at=[1.0, 0.5, 0.5], width=12, height=12 + i))
    return cams


def _refs(idx, cams, tfs):
    out = []
    for i, cam in enumerate(cams):
        out.append(L.sph_hoa_render(idx, cam, tfs[i % len(tfs)], 0.0, VMAX, STEP).clone())
    torch.cuda.synchronize()
    return out


def test_served_images_equal_single_renders():
    sc = H.tiny_scene()
    idx = sc.index()
    tfs = [torch.as_tensor(synth.transfer_function(seed=3), device="cuda"),
           torch.as_tensor(synth.transfer_function(seed=8), device="cuda")]
    cams = _cams()
    refs = _refs(idx, cams, tfs)
    big = synth.tiny_camera(256, 256)
    big_ref = L.sph_hoa_render(idx, big, tfs[0], 0.0, VMAX, STEP).clone()
    torch.cuda.synchronize()
    srv = L.Server(hbm_budget_bytes=1 << 30, lanes=1)
    try:
        slot = srv.add_index(idx)
        # a large request first keeps the lane busy while the small ones queue up behind it
        big_id, big_out = srv.submit(slot, big, tfs[0], 0.0, VMAX, STEP)
        ids = [None] * len(cams)
        outs = [None] * len(cams)

        def submitter(k):
            for i in range(k, len(cams), 3):
                ids[i], outs[i] = srv.submit(slot, cams[i], tfs[i % 2], 0.0, VMAX, STEP)

        th = [threading.Thread(target=submitter, args=(k,)) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        done, lat = srv.wait(big_id, 120.0)
        assert done and lat > 0
        assert torch.equal(big_out, big_ref)
        for i, cam in enumerate(cams):
            done, lat = srv.wait(ids[i], 120.0)
            assert done
            assert torch.equal(outs[i], refs[i]), cam
        st = srv.stats()
        assert st["completed"] == len(cams) + 1 and st["failed"] == 0 and st["queued"] == 0
        assert st["batches"] < st["completed"]  # requests shared launches
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    finally:
        srv.close()


def test_requests_arriving_mid_batch_overlap_running_work():
    """Continuous batching: a heavy request of one index is being rendered when small requests of
    two indices arrive; a second lane admits them at once (their work overlaps the running batch on
    the device, and they complete before it), and every image equals its single render bit for bit."""
    tiny = H.tiny_scene()
    ia = tiny.index()
    xyz, h, val = synth.clustered_particles(seed=12, n=200_000)
    heavy = H.Scene("wendland", 4, 3, 4096, xyz, h, val, 1e-3)
    ib = heavy.index()
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    persp = {"eye": [0.5, 0.5, -1.5], "look_at": [0.5, 0.5, 0.5], "up": [0.0, 1.0, 0.0], "fov_y_deg": 30.0,
             "ortho": 0, "ortho_half_extent": 0.0, "width": 512, "height": 512, "t_min": 1.0, "t_max": 3.0}
    # the heavy request: 1024^2 rays through the 200k clustered set, several times the small
    # requests' work even when their kernels wait for a slice of it to end
    big = dict(persp, width=1024, height=1024)
    vb, sb = 300.0, 2.0 / 512
    small_a = _cams()[:5]
    small_b = [dict(persp, width=32 + 8 * i, height=24, fov_y_deg=5.0 + i) for i in range(4)]
    big_ref = L.sph_hoa_render(ib, big, tf, 0.0, vb, sb).clone()
    refs_a = _refs(ia, small_a, [tf])
    refs_b = [L.sph_hoa_render(ib, c, tf, 0.0, vb, sb).clone() for c in small_b]
    torch.cuda.synchronize()
    srv = L.Server(hbm_budget_bytes=1 << 30, lanes=2)
    try:
        sa, sb_slot = srv.add_index(ia), srv.add_index(ib)
        big_id, big_out = srv.submit(sb_slot, big, tf, 0.0, vb, sb)
        subs_a = [srv.submit(sa, c, tf, 0.0, VMAX, STEP) for c in small_a]
        subs_b = [srv.submit(sb_slot, c, tf, 0.0, vb, sb) for c in small_b]
        lat_small = []
        for (rid, out), ref in zip(subs_a + subs_b, refs_a + refs_b):
            done, lat = srv.wait(rid, 120.0)
            assert done
            assert torch.equal(out, ref)
            lat_small.append(lat)
        done, lat_big = srv.wait(big_id, 120.0)
        assert done
        assert torch.equal(big_out, big_ref)
        st = srv.stats()
        assert st["lanes"] == 2 and st["completed"] == 1 + len(small_a) + len(small_b) and st["failed"] == 0
        assert st["overlapped_batches"] >= 1 and st["max_in_flight"] == 2, st
        print(f"small requests: max latency {max(lat_small):.1f} ms; heavy request: {lat_big:.1f} ms", flush=True)
        assert max(lat_small) < lat_big, (lat_small, lat_big)
    finally:
        srv.close()


def test_budget_admits_one_request_per_batch():
    sc = H.tiny_scene()
    idx = sc.index()
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    cams = _cams()[:6]
    refs = _refs(idx, cams, [tf])
    srv = L.Server(hbm_budget_bytes=1)  # nothing fits beside the head request
    try:
        slot = srv.add_index(idx)
        sub = [srv.submit(slot, c, tf, 0.0, VMAX, STEP) for c in cams]
        for (rid, out), ref in zip(sub, refs):
            assert srv.wait(rid, 120.0)[0]
            assert torch.equal(out, ref)
        st = srv.stats()
        assert st["batches"] == st["completed"] == len(cams)
    finally:
        srv.close()


def test_server_errors_and_timeouts():
    sc = H.tiny_scene()
    idx = sc.index()
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    srv = L.Server()
    try:
        slot = srv.add_index(idx)
        with pytest.raises(L.SphHoaError):
            srv.submit(slot + 5, synth.tiny_camera(8, 8), tf, 0.0, VMAX, STEP)
        with pytest.raises(L.SphHoaError):
            srv.submit(slot, dict(synth.tiny_camera(8, 8), t_min=2.0, t_max=1.0), tf, 0.0, VMAX, STEP)
        with pytest.raises(L.SphHoaError):
            srv.wait(12345, 0.0)
        rid, out = srv.submit(slot, synth.tiny_camera(64, 64), tf, 0.0, VMAX, STEP)
        done, _ = srv.wait(rid, 0.0)  # may or may not be finished yet
        if not done:
            done, _ = srv.wait(rid, 120.0)
        assert done
        with pytest.raises(L.SphHoaError):  # the id was released by the completed wait
            srv.wait(rid, 0.0)
    finally:
        srv.close()


def test_admission_limits_cancel_and_pause():
    import time

    sc = H.tiny_scene()
    idx = sc.index()
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    cams = _cams()[:4]
    refs = _refs(idx, cams, [tf])
    srv = L.Server()
    try:
        slot = srv.add_index(idx)
        srv.set_admission(max_queued=2)
        srv.pause(True)
        r0, _ = srv.submit(slot, cams[0], tf, 0.0, VMAX, STEP)
        r1, o1 = srv.submit(slot, cams[1], tf, 0.0, VMAX, STEP)
        with pytest.raises(L.SphHoaError) as e:  # two already wait
            srv.submit(slot, cams[2], tf, 0.0, VMAX, STEP)
        assert L.STATUS[e.value.status] == "E_BUSY"
        assert srv.cancel(r0)
        with pytest.raises(L.SphHoaError) as e:
            srv.wait(r0, 0.0)
        assert L.STATUS[e.value.status] == "E_CANCELLED"
        with pytest.raises(L.SphHoaError):  # the cancelled id was collected by its wait
            srv.cancel(r0)
        r2, o2 = srv.submit(slot, cams[2], tf, 0.0, VMAX, STEP)  # room again
        assert srv.stats()["queued"] == 2
        assert srv.wait(r1, 0.2)[0] is False and srv.stats()["completed"] == 0  # paused: nothing runs
        srv.pause(False)
        assert srv.wait(r1, 120.0)[0] and srv.wait(r2, 120.0)[0]
        assert torch.equal(o1, refs[1]) and torch.equal(o2, refs[2])
        # a request that already ran cannot be cancelled; its wait still reports it
        r3, o3 = srv.submit(slot, cams[3], tf, 0.0, VMAX, STEP)
        t0 = time.time()
        while srv.stats()["completed"] < 3 and time.time() - t0 < 60:
            time.sleep(0.01)
        assert not srv.cancel(r3)
        assert srv.wait(r3, 120.0)[0] and torch.equal(o3, refs[3])
        # one request larger than the per-request memory bound is refused outright
        srv.set_admission(max_queued=0, max_request_bytes=1000)
        with pytest.raises(L.SphHoaError) as e:
            srv.submit(slot, synth.tiny_camera(64, 64), tf, 0.0, VMAX, STEP)
        assert L.STATUS[e.value.status] == "E_OUT_OF_MEMORY"
        st = srv.stats()
        assert st["rejected"] == 2 and st["cancelled"] == 1 and st["completed"] == 3 and st["failed"] == 0
    finally:
        srv.close()


def test_destroy_drains_a_paused_queue():
    sc = H.tiny_scene()
    idx = sc.index()
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    cam = _cams()[1]
    ref = _refs(idx, [cam], [tf])[0]
    srv = L.Server()
    slot = srv.add_index(idx)
    srv.pause(True)
    _, out = srv.submit(slot, cam, tf, 0.0, VMAX, STEP)
    srv.close()  # renders what is queued, then stops
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
