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
