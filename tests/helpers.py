"""Shared helpers of the GPU tests: device transfer with padded pitches, random states."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_dev(a, pad=0):
    """float64 numpy -> float32 CUDA plane; pad > 0 gives a row pitch of W + pad elements."""
    a = np.asarray(a, dtype=np.float32)
    H, W = a.shape
    if pad:
        base = torch.zeros((H, W + pad), dtype=torch.float32, device=dev())
        t = base[:, :W]
        t.copy_(torch.from_numpy(a).to(dev()))
        return t
    return torch.from_numpy(a.copy()).to(dev())


def to_np(t):
    return t.detach().to("cpu").numpy().astype(np.float64)


def f32(a):
    """Round to float32 and back, so the oracle sees exactly the GPU's inputs."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def random_admm_state(rng, shape, beta):
    st = {}
    for k in ("u", "v"):
        st[k] = f32(rng.normal(scale=2.0, size=shape))
    for k in ("q1x", "q1y", "q2x", "q2y"):
        st[k] = f32(rng.uniform(-0.5, 0.5, size=shape))
    st["s"] = f32(rng.uniform(-0.05, 0.05, size=shape))
    if beta > 0:
        st["w"] = f32(rng.normal(scale=0.5, size=shape))
        st["px"] = f32(rng.uniform(-0.6, 0.6, size=shape))
        st["py"] = f32(rng.uniform(-0.6, 0.6, size=shape))
    else:
        st["w"] = np.zeros(shape)
        st["px"] = np.zeros(shape)
        st["py"] = np.zeros(shape)
    return st


def random_lin(rng, shape, beta):
    Ix = f32(rng.normal(0, 20, size=shape))
    Iy = f32(rng.normal(0, 20, size=shape))
    It = f32(rng.normal(0, 15, size=shape))
    at = float(np.float32(np.max(beta * beta + Ix * Ix + Iy * Iy)))
    return Ix, Iy, It, at


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0


def _oracle_job(args):
    from oracle import Params as OParams, solve_pair
    I0, I1, kw = args
    r = solve_pair(I0, I1, OParams(**kw))
    return r["u"], r["v"], (r["energy"], r["gap"])


def oracle_with_sensitivity(jobs, pool, probes=1):
    """Start the FP64 oracle on every (I0, I1, kwargs) job and on `probes` copies of its frames
    perturbed by independent 1e-7 relative noise (seeded), in `pool`.  Returns a callable
    get(timeout) -> [[ref, pert_1, ..., pert_probes] per job]."""
    rng = np.random.default_rng(123)
    work = []
    for I0, I1, kw in jobs:
        work.append((I0, I1, kw))
        for _ in range(probes):
            P0 = I0 * (1 + 1e-7 * rng.standard_normal(I0.shape))
            P1 = I1 * (1 + 1e-7 * rng.standard_normal(I1.shape))
            work.append((P0, P1, kw))
    fut = pool.map_async(_oracle_job, work)

    def get(timeout):
        r = fut.get(timeout=timeout)
        g = probes + 1
        return [r[g * k:g * (k + 1)] for k in range(len(jobs))]
    return get


def assert_conditioned(name, u, v, res, ref, perts):
    """Per-pixel bar 1e-4 px + 10 x the oracle's own response to perturbations of its input frames
    of the size of FP32 rounding (largest over the probes and over a 5 x 5 neighbourhood); energy /
    gap within 1e-6 / 1e-5 of the energy, widened likewise."""
    import scipy.ndimage
    ru, rv, (re, rgap) = ref
    resp = np.zeros_like(ru)
    de = dg = 0.0
    for pu, pv, (pe, pgap) in perts:
        resp = np.maximum(resp, np.maximum(np.abs(pu - ru), np.abs(pv - rv)))
        de = max(de, abs(pe - re))
        dg = max(dg, abs(pgap - rgap))
    d = np.maximum(np.abs(u - ru), np.abs(v - rv))
    sens = scipy.ndimage.maximum_filter(resp, size=5, mode="nearest")
    print(f"[parity] {name}: max {d.max():.3e} p99.9 {np.quantile(d, 0.999):.3e} mean {d.mean():.3e}; "
          f"sensitivity max {sens.max():.2e} ({len(perts)} probes); energy {res['energy']:.4f} vs {re:.4f}", flush=True)
    bad = d > 1e-4
    for i, j in list(zip(*np.where(bad)))[:20]:
        print(f"[parity] {name}: pixel ({i},{j}) |d| {d[i, j]:.2e} sensitivity {sens[i, j]:.2e} "
              f"oracle u,v {ru[i, j]:.4f},{rv[i, j]:.4f}", flush=True)
    assert np.all(d <= 1e-4 + 10.0 * sens), float((d - 1e-4 - 10.0 * sens).max())
    assert abs(res["energy"] - re) <= 1e-6 * re + 10.0 * de, (res["energy"], re, de)
    assert abs(res["gap"] - rgap) <= 1e-5 * re + 10.0 * dg, (res["gap"], rgap, dg)
