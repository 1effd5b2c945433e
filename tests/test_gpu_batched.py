"""GPU parity of the ragged batch: one persistent launch gives each image the
same outputs as the plain call on that image (and the oracle's masks)."""
import numpy as np
import pytest
import torch

import oracle
from docgen import gen_document, gen_batch, batch_specs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1905_13038_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def plain(bz, img, p):
    if p.get("method", "sauvola") == "sauvola":
        return bz.sauvola(img, p["h"], p["w"], k=p["k"], R=p.get("R", 128.0), stats=p.get("stats", True))
    return bz.niblack(img, p["h"], p["w"], k=p["k"], stats=p.get("stats", True))


def same(a, b):
    if a is None or b is None:
        return a is None and b is None
    return torch.equal(a, b)


def small_batch():
    rng = np.random.default_rng(7)
    imgs, params = [], []
    shapes = [(384, 512), (1, 1), (37, 4100), (700, 257), (64, 9000), (5, 3), (1000, 1024),
              (333, 1025), (129, 130), (2048, 300), (17, 2000), (256, 4096)]
    for i, (H, W) in enumerate(shapes):
        imgs.append(dev(gen_document(H, W, 100 + i, noise=10, stain=True)))
        win = int(rng.integers(1, 60)) | 1
        params.append(dict(h=win, w=int(rng.integers(1, 80)), k=float(np.float32(rng.uniform(0.2, 0.5))),
                           R=128.0, method="sauvola" if i % 3 else "niblack", stats=(i % 4 != 1)))
    # one unaligned view (odd base offset and stride)
    base = dev(gen_document(300, 701, 999, noise=10))
    imgs.append(base[:, 1:700])
    params.append(dict(h=31, w=31, k=0.4, R=120.0, method="sauvola"))
    return imgs, params


def test_batch_equals_plain_calls_and_oracle(bz):
    imgs, params = small_batch()
    out = bz.sauvola_batched(imgs, params)
    torch.cuda.synchronize()
    for img, p, (mask, m, s) in zip(imgs, params, out):
        pm, pmean, pstd = plain(bz, img, p)
        assert same(mask, pm) and same(m, pmean) and same(s, pstd), p
        host = img.cpu().numpy()
        if p["method"] == "sauvola":
            ref = oracle.sauvola(host, p["h"], p["w"], k=p["k"], R=p["R"])
        else:
            ref = oracle.niblack(host, p["h"], p["w"], k=p["k"])
        assert np.array_equal(mask.cpu().numpy(), ref["mask"]), p


def test_batch_of_one_and_order_invariance(bz):
    imgs, params = small_batch()
    one = bz.sauvola_batched(imgs[:1], params[:1])[0]
    pm = plain(bz, imgs[0], params[0])
    assert all(same(a, b) for a, b in zip(one, pm))
    perm = list(range(len(imgs)))[::-1]
    a = bz.sauvola_batched(imgs, params)
    b = bz.sauvola_batched([imgs[i] for i in perm], [params[i] for i in perm])
    for i, j in enumerate(perm):
        assert all(same(x, y) for x, y in zip(a[j], b[i]))


@pytest.mark.parametrize("strip", [1, 3, 16, 200])
def test_strip_choice_does_not_change_results(bz, strip):
    imgs, params = small_batch()
    ref = bz.sauvola_batched(imgs, params)
    got = bz.sauvola_batched(imgs, params, strips=[strip] * len(imgs))
    for x, y in zip(ref, got):
        assert all(same(p, q) for p, q in zip(x, y))


def test_graph_replays(bz):
    imgs, params = small_batch()
    plan = bz.BatchPlan(imgs, params)
    plan.capture()
    torch.cuda.synchronize()
    refs = [plain(bz, i, p) for i, p in zip(imgs, params)]
    for rep in range(4):
        for mask, m, s in plan.outputs():  # clear eagerly between replays
            mask.zero_()
            if m is not None:
                m.zero_()
                s.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        plan.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for (mask, m, s), (rm, rmean, rstd) in zip(plan.outputs(), refs):
            assert same(mask, rm) and same(m, rmean) and same(s, rstd), rep


def test_full_ragged_batch_256(bz):
    # the 256-page ragged workload: every page equals its plain call on the
    # device; eight pages are also checked against the oracle
    specs = batch_specs()
    print("generating 256 pages", flush=True)
    pages = gen_batch(specs, workers=8)
    imgs = [dev(p) for p in pages]
    params = [dict(h=d["h"], w=d["w"], k=d["k"], R=d["R"], method="sauvola") for d in specs]
    plan = bz.BatchPlan(imgs, params)
    plan.run()
    torch.cuda.synchronize()
    print("batched run done", flush=True)
    for i, (img, p) in enumerate(zip(imgs, params)):
        pm, pmean, pstd = plain(bz, img, p)
        mask, m, s = plan.outputs()[i]
        assert same(mask, pm) and same(m, pmean) and same(s, pstd), i
        del pm, pmean, pstd
    for i in range(0, 256, 32):
        d = specs[i]
        ref = oracle.sauvola(pages[i], d["h"], d["w"], k=d["k"], R=d["R"])
        assert np.array_equal(plan.outputs()[i][0].cpu().numpy(), ref["mask"]), i


def test_autotuned_strips(bz):
    from paper_1905_13038_amd import tune
    table = tune.autotune(count=4, H=256, W=320, candidates=(16, 40), classes=(15, 31), reps=1,
                          cache_path=None)
    assert set(table) == {15, 31} and all(v in (16, 40) for v in table.values())
    rng = np.random.default_rng(7)
    imgs = [dev(gen_document(int(rng.integers(200, 400)), int(rng.integers(200, 400)), 70 + i,
                             noise=10.0, stain=True)) for i in range(5)]
    params = [{"h": h, "w": h, "k": 0.4} for h in (11, 15, 21, 29, 31)]
    plan = bz.BatchPlan(imgs, params, strips=tune.strips_for(params, table))
    plan.run()
    torch.cuda.synchronize()
    for img, p, (mk, m, s) in zip(imgs, params, plan.outputs()):
        mk0, m0, s0 = plain(bz, img, p)
        assert torch.equal(mk, mk0) and torch.equal(m, m0) and torch.equal(s, s0)


def test_in_situ_tuning_and_replan(bz):
    # autotune_plan re-plans the batch on its own outputs for each trial and
    # leaves it on the chosen strips; the results equal the plain calls
    from paper_1905_13038_amd import tune
    imgs, params = small_batch()
    plan = bz.BatchPlan(imgs, params)
    table = tune.autotune_plan(plan, params, candidates=(8, 64), reps=1)
    assert set(table) <= {tune.window_class(int(p["h"])) for p in params}
    assert all(v in (8, 64) for v in table.values())
    for strips in (None, [5] * len(imgs)):
        plan.replan(strips)
        for mask, m, s in plan.outputs():
            mask.zero_()
        plan.run()
        torch.cuda.synchronize()
        for img, p, (mk, m, s) in zip(imgs, params, plan.outputs()):
            mk0, m0, s0 = plain(bz, img, p)
            assert same(mk, mk0) and same(m, m0) and same(s, s0)


def test_plan_outputs_rows_on_64_byte_boundaries(bz):
    # BatchPlan pads its output rows so that each row starts on a 64-byte
    # boundary; the values match plain calls with contiguous outputs
    rng = np.random.default_rng(11)
    imgs = [dev(gen_document(int(rng.integers(60, 200)), W, 90 + i, noise=10.0, stain=True))
            for i, W in enumerate((37, 64, 101, 250))]
    params = [{"h": 9, "w": 13, "k": 0.3, "method": "sauvola"},
              {"h": 15, "w": 15, "k": 0.2, "method": "niblack"},
              {"h": 5, "w": 3, "k": 0.5}, {"h": 31, "w": 21, "k": 0.4}]
    plan = bz.BatchPlan(imgs, params)
    plan.run()
    torch.cuda.synchronize()
    for img, p, (mk, m, s) in zip(imgs, params, plan.outputs()):
        assert mk.shape == img.shape and m.shape == img.shape
        assert mk.stride(0) % 64 == 0 and (4 * m.stride(0)) % 64 == 0 and m.stride(0) == s.stride(0)
        assert mk.data_ptr() % 64 == 0 and m.data_ptr() % 64 == 0 and s.data_ptr() % 64 == 0
        mk0, m0, s0 = plain(bz, img, p)
        assert torch.equal(mk, mk0) and torch.equal(m, m0) and torch.equal(s, s0)
