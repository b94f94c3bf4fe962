"""The serving session on the GPU: every request's frame equals the frame
ssr_shade renders alone, while requests of mixed size run concurrently under
a device-memory budget that binds."""

import numpy as np
import pytest
import torch

import scenes
from scenes import quantise_gbuffer

pytestmark = pytest.mark.gpu


def _upload(sc, dtype, dev):
    t = {"depth": torch.from_numpy(sc.depth).to(dev), "env": torch.from_numpy(sc.env).to(dev)}
    if dtype == "f32":
        for k in ("normal_rough", "albedo_metal", "radiance"):
            t[k] = torch.from_numpy(getattr(sc, k)).to(dev)
    else:
        bits, _ = quantise_gbuffer(sc, dtype)
        tdt = torch.float16 if dtype == "f16" else torch.bfloat16
        for k in ("normal_rough", "albedo_metal", "radiance"):
            t[k] = torch.from_numpy(bits[k].view(np.int16)).to(dev).view(tdt)
    return t


def _scenes():
    # three resolutions and storage types of the 1080p scene's object mix
    out = []
    for (w, h, dt, seed) in ((96, 64, "f16", 21), (160, 90, "f32", 22), (203, 117, "f16", 23)):
        out.append((scenes.make_scene("c2", seed=seed, width=w, height=h), dt))
    return out


def _params(sc, spp, seed, march="hiz"):
    p = dict(sc.params, spp=spp, seed=seed, frame=seed % 7)
    if march == "linear":
        p.update(march=0, max_steps=32, max_dist=4.0)
    return p


def _intervals_overlap(a, b):
    return a["t_admit"] < b["t_done"] and b["t_admit"] < a["t_done"]


@pytest.mark.parametrize("graphs", [True, False])
def test_results_in_the_mix_equal_results_alone(graphs):
    """Each request's frame equals ssr_shade alone, bit for bit: with frames
    replayed from each slot's graphs (every shape class is built once per
    slot, then replayed with new node parameters: 18 requests over 3 sizes
    and 2 march modes on 3 slots) and with frames launched directly."""
    from paper_2504_01358_amd import ssr
    dev = torch.device("cuda", 0)
    ctx = ssr.Context(0)
    scs = _scenes()
    ups = [_upload(sc, dt, dev) for sc, dt in scs]
    sess = ssr.Session(0, hbm_budget_bytes=256 << 20, max_slots=3, max_bypass=2, graphs=graphs)
    ids = [sess.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                          u["radiance"], u["env"]) for (sc, _), u in zip(scs, ups)]
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(18):
        s = int(rng.integers(0, len(scs)))
        spp = int(rng.choice([1, 4, 16, 64]))
        march = "linear" if k % 6 == 5 else "hiz"
        # (odd requests: a seed whose high word is set, carried into the graph nodes)
        seed = 1000 + k + ((0x9E3779B9 << 32) if k % 2 else 0)
        reqs.append((s, _params(scs[s][0], spp, seed, march)))
    tickets = [sess.submit(ids[s], p) for s, p in reqs]
    results = [sess.wait(t) for t, _ in tickets]
    assert all(r["status"] == 0 for r in results)
    assert all(r["t_submit"] <= r["t_admit"] <= r["t_done"] for r in results)
    # work really ran side by side
    assert any(_intervals_overlap(a, b) for i, a in enumerate(results) for b in results[i + 1:])
    for (s, p), (t, out) in zip(reqs, tickets):
        sc, _ = scs[s]
        u = ups[s]
        alone = ctx.shade(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                          u["radiance"], u["env"], p)
        torch.cuda.synchronize()
        assert torch.equal(out, alone), (s, p["spp"], p["march"])
    st = sess.stats()
    assert st["running"] == 0 and st["waiting"] == 0 and st["arena_used"] == 0
    assert st["completed"] == len(reqs)
    sess.close()
    ctx.close()


def test_budget_binds_admission():
    """With room for one large workspace at a time, large requests never
    overlap each other, small ones run beside them, and the arena is never
    over-committed."""
    from paper_2504_01358_amd import ssr
    dev = torch.device("cuda", 0)
    sc = scenes.make_scene("c2", seed=31, width=320, height=180)
    u = _upload(sc, "f16", dev)
    probe = ssr.Session(0, hbm_budget_bytes=1 << 30, max_slots=4)
    sid = probe.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                          u["radiance"], u["env"])
    big_p, small_p = _params(sc, 64, 1), _params(sc, 1, 2)
    big, small = probe.request_bytes(sid, big_p), probe.request_bytes(sid, small_p)
    scene_bytes = probe.stats()["scene_bytes"]
    probe.close()
    budget = scene_bytes + big + big // 2
    sess = ssr.Session(0, hbm_budget_bytes=budget, max_slots=4, max_bypass=8)
    sid = sess.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                         u["radiance"], u["env"])
    kinds = ["big", "small", "small", "big", "small", "big", "small", "small", "big", "small"]
    tickets = [sess.submit(sid, dict(big_p if k == "big" else small_p, seed=10 + i))
               for i, k in enumerate(kinds)]
    res = [sess.wait(t) for t, _ in tickets]
    arena = budget - scene_bytes
    assert all(r["status"] == 0 for r in res)
    bigs = [r for r, k in zip(res, kinds) if k == "big"]
    assert not any(_intervals_overlap(a, b) for i, a in enumerate(bigs) for b in bigs[i + 1:])
    events = sorted([(r["t_admit"], r["workspace_bytes"]) for r in res]
                    + [(r["t_done"], -r["workspace_bytes"]) for r in res], key=lambda e: (e[0], e[1]))
    held = peak = 0
    for _, b in events:
        held += b
        peak = max(peak, held)
    assert peak <= arena
    assert any(_intervals_overlap(a, b) for a in bigs for b, k in zip(res, kinds) if k == "small")
    # a request that can never fit is refused at submission
    with pytest.raises(ssr.SSRError) as e:
        sess.submit(sid, dict(big_p, spp=4096))
    assert e.value.status == -6
    sess.close()


def test_session_errors_and_lifecycle():
    from paper_2504_01358_amd import ssr
    dev = torch.device("cuda", 0)
    sc = scenes.make_scene("c1", width=32, height=24)
    u = _upload(sc, "f32", dev)
    sess = ssr.Session(0, hbm_budget_bytes=64 << 20, max_slots=2)
    sid = sess.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                         u["radiance"], u["env"])
    for bad in (dict(spp=0), dict(march=5), dict(thickness=-1.0)):
        with pytest.raises(ssr.SSRError):
            sess.submit(sid, dict(sc.params, **bad))
    t, out = sess.submit(sid, sc.params)
    r = sess.wait(t)
    assert r["status"] == 0
    with pytest.raises(ssr.SSRError) as e:       # retired
        sess.poll(t)
    assert e.value.status == -8
    with pytest.raises(ssr.SSRError) as e:       # serving: no more scenes
        sess.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                       u["radiance"], u["env"])
    assert e.value.status == -7
    # stop with work queued and running: waiting requests are dropped cleanly
    for k in range(20):
        sess.submit(sid, dict(sc.params, spp=64, seed=k))
    sess.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("graphs", [True, False])
def test_split_units_equal_whole_tiles(graphs):
    """A 1280x720 frame (14,400 tiles for at most a few thousand resident
    waves) is traced by ssr_shade with its tiles handed out in parts of their
    samples, and by a serving session with whole tiles (a session splits only
    frames with fewer tiles than waves): which wave marches which ray must not
    change the image, bit for bit."""
    from paper_2504_01358_amd import ssr
    dev = torch.device("cuda", 0)
    ctx = ssr.Context(0)
    sc = scenes.make_scene("c2", seed=41, width=1280, height=720)
    u = _upload(sc, "f32", dev)
    sess = ssr.Session(0, hbm_budget_bytes=1 << 30, max_slots=1, max_bypass=0, graphs=graphs)
    sid = sess.add_scene(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"],
                         u["radiance"], u["env"])
    p = dict(sc.params, seed=9, frame=2)
    t, out = sess.submit(sid, p)
    r = sess.wait(t)
    alone = ctx.shade(sc.camera, u["depth"], u["normal_rough"], u["albedo_metal"], u["radiance"],
                      u["env"], p)
    torch.cuda.synchronize()
    assert r["status"] == 0
    assert torch.equal(out, alone)
    sess.close()
    ctx.close()
