"""Learned row filter on the MI355X against the FP64 oracle: each layer
kernel (forward, backward-data, backward-weight) over every supported channel
pair and ragged row lengths, the cosine weight, the loss and Adam kernels, the
whole network, a full training gradient through BP and its transpose, and a
short training run that must beat the ramp filter on held-out phantoms."""
import numpy as np
import pytest

import oracle
from oracle import learned as ol
from oracle import geometry as og
from oracle import phantom as oph
import workloads as wl
from helpers import log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd import learned as L  # noqa: E402
from paper_2104_13248_amd.autograd import Geometry  # noqa: E402

TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


PAIRS = [(1, 32), (32, 32), (32, 1), (1, 1)]
LENS = [1, 7, 130, 256, 257, 600]


@pytest.mark.parametrize("cin,cout", PAIRS)
@pytest.mark.parametrize("n", LENS)
def test_conv_forward_parity(cin, cout, n):
    seed = 100 * cin + cout + 7 * n
    rows = 5
    x = wl.gaussian(seed, (rows, cin, n))
    w = wl.gaussian(seed + 1, (cout, cin, 9))
    b = wl.gaussian(seed + 2, (cout,))
    got = host(L.conv1d_forward(dev(x), dev(w), dev(b)))
    ref = ol.conv(x.astype(np.float64), w.astype(np.float64), b.astype(np.float64))
    assert rel(got, ref) <= TOL32


@pytest.mark.parametrize("cin,cout", PAIRS)
def test_conv_forward_epilogue(cin, cout):
    """relu, mask, alpha and the residual addend (also accumulated in place)."""
    seed = 300 + 10 * cin + cout
    rows, n = 4, 301
    x = wl.gaussian(seed, (rows, cin, n))
    w = wl.gaussian(seed + 1, (cout, cin, 9))
    b = wl.gaussian(seed + 2, (cout,))
    mask = wl.gaussian(seed + 3, (rows, cout, n))
    add = wl.gaussian(seed + 4, (rows, cout, n))
    alpha = 0.37
    out = dev(add)
    L.conv1d_forward(dev(x), dev(w), dev(b), mask=dev(mask), add=out, alpha=alpha, relu=True,
                     out=out)
    y = ol.relu(ol.conv(x.astype(np.float64), w.astype(np.float64), b.astype(np.float64)))
    ref = alpha * y * (mask > 0) + add
    assert rel(host(out), ref) <= TOL32


@pytest.mark.parametrize("cin,cout", PAIRS)
@pytest.mark.parametrize("n", [3, 256, 517])
def test_conv_backward_data_parity(cin, cout, n):
    seed = 500 + 100 * cin + cout + n
    rows = 6
    g = wl.gaussian(seed, (rows, cout, n))
    w = wl.gaussian(seed + 1, (cout, cin, 9))
    mask = wl.gaussian(seed + 2, (rows, cin, n))
    got = host(L.conv1d_backward_data(dev(g), dev(w), mask=dev(mask)))
    ref = ol.conv_backward_data(g.astype(np.float64), w.astype(np.float64)) * (mask > 0)
    assert rel(got, ref) <= TOL32


@pytest.mark.parametrize("cin,cout", PAIRS)
@pytest.mark.parametrize("rows,n", [(1, 5), (37, 129), (2100, 64), (600, 512)])
def test_conv_backward_weight_parity(cin, cout, rows, n):
    seed = 700 + 100 * cin + cout + rows + n
    x = wl.gaussian(seed, (rows, cin, n))
    g = wl.gaussian(seed + 1, (rows, cout, n))
    gw0 = wl.gaussian(seed + 2, (cout, cin, 9))
    gb0 = wl.gaussian(seed + 3, (cout,))
    gw, gb = dev(gw0), dev(gb0)
    L.conv1d_backward_weight(dev(x), dev(g), gw, gb)
    rw, rb = ol.conv_backward_weight(x.astype(np.float64), g.astype(np.float64))
    assert rel(host(gw), rw + gw0) <= TOL32
    assert rel(host(gb), rb + gb0) <= TOL32


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 1), (1, 32)])
def test_conv_backward_weight_deterministic(cin, cout):
    """The weight gradients of the 32-channel layers are summed per block and
    then across blocks in a fixed order: two calls agree bitwise."""
    rows, n = 300, 512
    x = dev(wl.gaussian(950 + cin, (rows, cin, n)))
    g = dev(wl.gaussian(951 + cout, (rows, cout, n)))
    out = []
    for _ in range(2):
        gw = torch.zeros((cout, cin, 9), dtype=torch.float32, device="cuda")
        gb = torch.zeros((cout,), dtype=torch.float32, device="cuda")
        L.conv1d_backward_weight(x, g, gw, gb)
        out.append((host(gw), host(gb)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_cosine_weight_parity():
    scan = dict(wl.CONFIGS["c5"]["scan"], u_off=3.0, v_off=-2.5)
    raw = wl.gaussian(900, (3, 40, 77))
    got = host(L.cosine_weight(dev(raw), scan))
    ref = ol.cosine_weight(raw.astype(np.float64), scan)
    assert rel(got, ref) <= 1e-6


def test_sqerr_and_adam_parity():
    a = wl.gaussian(910, (1000003,))
    b = wl.gaussian(911, (1000003,))
    grad = torch.empty(a.shape, dtype=torch.float32, device="cuda")
    loss = L.sqerr(dev(a), dev(b), grad, grad_scale=0.5)
    rl, _ = ol.sqerr(a, b)
    assert abs(float(host(loss)[0]) - rl) <= 1e-5 * rl
    assert rel(host(grad), 0.5 * (a.astype(np.float64) - b)) <= 1e-7

    p0 = wl.gaussian(920, (2000,)).astype(np.float64)
    gs = [wl.gaussian(921 + t, (2000,)).astype(np.float64) for t in range(5)]
    p, m, v = dev(p0), torch.zeros(2000, device="cuda"), torch.zeros(2000, device="cuda")
    rp, rm, rv = p0.copy(), np.zeros(2000), np.zeros(2000)
    # the kernel takes its hyper-parameters as float32: give the oracle those values
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    hp = dict(lr=f32(1e-2), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    for t in range(1, 6):
        L.adam_step(p, dev(gs[t - 1]), m, v, t, 1e-2)
        rp, rm, rv = ol.adam(rp, gs[t - 1], rm, rv, t, **hp)
    assert rel(host(p) - p0, rp - p0) <= 1e-5
    assert rel(host(m), rm) <= 1e-6 and rel(host(v), rv) <= 1e-6


def small_case(seed=0, np_views=12, nh=40, nw=72, shape=(24, 28, 32)):
    cfg = wl.CONFIGS["c5"]
    scan = cfg["scan"]
    # same physical detector and FOV as the full workload, coarser sampling
    scale_det = cfg["nw"] / nw
    scan = dict(scan, du=scan["du"] * scale_det, dv=scan["dv"] * cfg["nh"] / nh)
    voxel = tuple(v * cfg["shape"][0] / shape[0] for v in cfg["voxel"])
    ell = wl.config_ellipsoids(cfg, seed)
    raw = oph.line_integrals(ell, scan, np_views, nh, nw).astype(np.float32)
    mats = og.scan_matrices(scan, np_views, nh, nw)
    geom = Geometry(tuple(shape), voxel, fdk.scan_matrices(scan, np_views, nh, nw), nh, nw)
    return scan, raw, mats, voxel, geom


def perturbed_params(seed):
    p = ol.init_params(seed, input_std=10.0, residual=False)
    rng = np.random.default_rng(seed)
    p["b1"] = 0.1 * rng.standard_normal(32)
    p["b2"] = 0.1 * rng.standard_normal(32)
    p["w3"] *= 0.05
    # float32-representable, so both sides start from the same numbers
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


@pytest.mark.parametrize("residual", [True, False])
def test_network_forward_parity(residual):
    scan, raw, mats, voxel, geom = small_case(1)
    p = perturbed_params(2)
    f = L.LearnedFilter("cuda", params=p, residual=residual)
    got = host(f.forward(dev(raw), scan))
    q = ol.cosine_weight(raw.astype(np.float64), scan)
    ramp = oracle.fdk_filter(raw.astype(np.float64), scan) if residual else None
    npv, nh, nw = raw.shape
    ref, _ = ol.net_forward(q.reshape(-1, nw), p, scan["arc"] / (2 * npv),
                            ramp.reshape(-1, nw) if residual else None)
    e = rel(got.reshape(-1, nw), ref)
    log("net forward rel-L2", e)
    assert e <= TOL32


def test_training_gradient_parity():
    """Gradient of mean((BP(filter(raw)) - target)^2) with respect to every
    parameter, through the HIP BP, its transpose and the layer kernels, against
    the oracle chain (oracle filter, oracle BP, oracle FP, oracle net)."""
    scan, raw, mats, voxel, geom = small_case(3)
    p = perturbed_params(4)
    target = wl.gaussian(930, geom.shape).astype(np.float64) * 0.01
    f = L.LearnedFilter("cuda", params=p, residual=True)
    f.grad.zero_()
    loss = f.loss_and_grad(dev(raw), dev(target), scan, geom)
    got = {k: host(v) for k, v in f.g.items()}

    npv, nh, nw = raw.shape
    alpha = scan["arc"] / (2 * npv)
    q = ol.cosine_weight(raw.astype(np.float64), scan).reshape(-1, nw)
    ramp = oracle.fdk_filter(raw.astype(np.float64), scan).reshape(-1, nw)
    y, cache = ol.net_forward(q, p, alpha, ramp)
    # the filtered stack is stored as float32 on both sides (the back-projector's input type)
    vol = oracle.backproject(y.reshape(npv, nh, nw).astype(np.float32), mats, geom.shape, voxel)
    rl, gvol = ol.sqerr(vol, target)
    gy = oracle.forwardproject(gvol, mats, nh, nw, voxel)
    ref = ol.net_backward(gy.reshape(-1, nw), p, alpha, cache)
    assert abs(float(host(loss)[0]) - rl) <= 1e-5 * rl
    for k in ref:
        e = rel(got[k], ref[k])
        log("grad", k, "rel-L2", e)
        assert e <= 1e-4, k


def test_checkpoint_roundtrip(tmp_path):
    scan, raw, mats, voxel, geom = small_case(5)
    f = L.LearnedFilter("cuda", params=perturbed_params(6), residual=True)
    target = torch.zeros(geom.shape, device="cuda")
    f.train_step(dev(raw), target, scan, geom, 1e-3)
    path = str(tmp_path / "ck.npz")
    f.save(path, next_phantom=17, seed=5000)
    g, meta = L.LearnedFilter.load(path)
    assert meta == {"next_phantom": 17, "seed": 5000} and g.t == f.t == 1
    for a, b in ((f.flat, g.flat), (f.m, g.m), (f.v, g.v)):
        assert torch.equal(a, b)


def test_short_training_beats_ramp_on_held_out():
    """Residual filter trained for a few dozen steps on 12-view scans against
    96-view ramp-FDK targets: lower held-out error than the plain ramp filter
    (which is where training starts)."""
    cfg = wl.CONFIGS["c5"]
    sparse, dense = 12, 96
    shape, nh, nw = (32, 32, 32), 48, 64
    base = dict(cfg["scan"])
    scan = dict(base, du=base["du"] * cfg["nw"] / nw, dv=base["dv"] * cfg["nh"] / nh)
    voxel = tuple(v * cfg["shape"][0] / shape[0] for v in cfg["voxel"])
    g_sparse = Geometry(shape, voxel, fdk.scan_matrices(scan, sparse, nh, nw), nh, nw)
    g_dense = Geometry(shape, voxel, fdk.scan_matrices(scan, dense, nh, nw), nh, nw)

    def scan_pair(i):
        ell = wl.config_ellipsoids(cfg, i)
        raw_s = torch.zeros((sparse, nh, nw), device="cuda")
        fdk.phantom_project(ell, scan, raw_s)
        raw_d = torch.zeros((dense, nh, nw), device="cuda")
        fdk.phantom_project(ell, scan, raw_d)
        tgt = torch.zeros(shape, device="cuda")
        fdk.backproject(tgt, fdk.fdk_filter(raw_d, scan), g_dense.mats, voxel)
        return raw_s, tgt

    train = [scan_pair(i) for i in range(8)]
    held = [scan_pair(100 + i) for i in range(4)]
    std = float(torch.cat([L.cosine_weight(r, scan).flatten() for r, _ in train]).std())
    f = L.LearnedFilter("cuda", residual=True, seed=1, input_std=std)

    def held_err():
        num = den = 0.0
        for raw_s, tgt in held:
            v = f.reconstruct(raw_s, scan, g_sparse)
            num += float(((v - tgt) ** 2).sum())
            den += float((tgt ** 2).sum())
        return (num / den) ** 0.5

    e0 = held_err()
    for it in range(48):
        raw_s, tgt = train[it % len(train)]
        f.train_step(raw_s, tgt, scan, g_sparse, lr=2e-3)
    e1 = held_err()
    log("held-out rel-L2 ramp %.4f learned %.4f" % (e0, e1))
    assert e1 < 0.95 * e0


def test_training_driver_end_to_end():
    """The training command at an eighth of C5's sampling (32^3, 64^2
    detector, 12-view scans against 96-view targets): six steps with the
    cosine learning-rate schedule, held-out evaluation before and after,
    finite results, and the summary's bookkeeping."""
    import math
    from paper_2104_13248_amd import train_learned
    s = train_learned.main(["--scale", "8", "--phantoms", "6", "--held-out", "2",
                            "--views", "12", "--target-views", "96", "--log-every", "3"])
    log("driver summary", {k: s[k] for k in ("ramp_rel_l2", "learned_rel_l2")})
    assert s["steps"] == 6 and s["shape"] == [32, 32, 32] and s["detector"] == [64, 64]
    assert s["ramp_rel_l2"] == s["ramp_rel_l2_before"] == s["learned_rel_l2_before"]
    assert math.isfinite(s["learned_rel_l2"]) and 0.0 < s["learned_rel_l2"] < 2.0 * s["ramp_rel_l2"]
    assert s["learned_ms"] > 0.0 and s["ramp_ms"] > 0.0
