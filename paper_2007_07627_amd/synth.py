"""Seeded synthetic scans for registration workloads.

Stand-ins for the paper's scan datasets (which are not available): surfaces
with analytic normals, partial overlap, uniform outliers, Gaussian noise and a
bounded random rigid motion, as in the paper's synthetic experiments (Sec. 6).
Everything is generated in FP64 with numpy's PCG64 and rounded to FP32 once.

This module holds no registration arithmetic: it only produces inputs and the
ground-truth motion. Both the GPU tests and the CPU oracle consume it.
"""
from __future__ import annotations

import math

import numpy as np


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    """Seed = 1000 * config + pair index."""
    return np.random.Generator(np.random.PCG64(1000 * config + index))


# --------------------------------------------------------------------------
# Surfaces
# --------------------------------------------------------------------------

def bumpy_sphere(rng, n, zmin=-1.0, zmax=1.0):
    """Points r(theta, phi) * u on the surface r = 1 + 0.1 sin(3 theta) sin(4 phi),
    directions uniform on the sphere restricted to zmin <= u_z <= zmax, with the
    analytic outward unit normal."""
    z = rng.uniform(zmin, zmax, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = np.arccos(np.clip(z, -1.0, 1.0))
    u = np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)
    r = 1.0 + 0.1 * np.sin(3 * th) * np.sin(4 * phi)
    pts = u * r[:, None]
    r_th = 0.3 * np.cos(3 * th) * np.sin(4 * phi)
    # r_phi / sin(theta) with sin(3t)/sin(t) = 3 - 4 sin^2 t (finite at the poles)
    r_ph_over_st = 0.4 * (3.0 - 4.0 * st * st) * np.cos(4 * phi)
    e_th = np.stack([z * np.cos(phi), z * np.sin(phi), -st], axis=1)
    e_ph = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    nrm = u - (r_th / r)[:, None] * e_th - (r_ph_over_st / r)[:, None] * e_ph
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


class HeightField:
    """z = 0.05 * sum_k sin(a_k x + b_k y), 8 seeded terms, a_k, b_k ~ U[-2pi, 2pi]."""

    def __init__(self, rng, terms=8):
        self.a = rng.uniform(-2 * math.pi, 2 * math.pi, terms)
        self.b = rng.uniform(-2 * math.pi, 2 * math.pi, terms)

    def sample(self, rng, n, xr=(-1.0, 1.0), yr=(-1.0, 1.0)):
        x = rng.uniform(xr[0], xr[1], n)
        y = rng.uniform(yr[0], yr[1], n)
        arg = np.outer(x, self.a) + np.outer(y, self.b)
        z = 0.05 * np.sin(arg).sum(axis=1)
        zx = 0.05 * (np.cos(arg) * self.a).sum(axis=1)
        zy = 0.05 * (np.cos(arg) * self.b).sum(axis=1)
        pts = np.stack([x, y, z], axis=1)
        nrm = np.stack([-zx, -zy, np.ones_like(zx)], axis=1)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        return pts, nrm


# --------------------------------------------------------------------------
# Motions and corruption
# --------------------------------------------------------------------------

def random_motion(rng, max_angle_deg, max_trans):
    """Rotation: angle uniform in [0, max], axis uniform on S^2 (unit quaternion
    to matrix). Translation: direction uniform, length uniform in [0, max]."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = math.radians(max_angle_deg) * rng.uniform()
    w = math.cos(ang / 2)
    x, y, z = axis * math.sin(ang / 2)
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    t = d * max_trans * rng.uniform()
    return R, t


def bbox_diag(pts):
    return float(np.linalg.norm(pts.max(axis=0) - pts.min(axis=0)))


def _apply(R, t, pts):
    return pts @ R.T + t


def _gt(R, t):
    """Ground truth mapping the moved source back onto the target: (R^T, -R^T t)."""
    T = np.eye(4)
    T[:3, :3] = R.T
    T[:3, 3] = -R.T @ t
    return T


def _replace_outliers(rng, src, frac):
    if frac <= 0:
        return src
    m = src.shape[0]
    k = int(round(frac * m))
    sel = rng.choice(m, size=k, replace=False)
    lo, hi = src.min(axis=0), src.max(axis=0)
    src = src.copy()
    src[sel] = rng.uniform(lo, hi, size=(k, 3))
    return src


def _pack(P, Q, Qn, T_gt, diag, **kw):
    d = dict(P=np.ascontiguousarray(P, np.float32), Q=np.ascontiguousarray(Q, np.float32),
             Qn=None if Qn is None else np.ascontiguousarray(Qn, np.float32),
             T_gt=T_gt, diag=diag)
    d.update(kw)
    return d


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def fast_icp_pair(rng, n=4096, max_angle=30.0, noise=1e-3):
    """Same points on both sides: target N = n on the bumpy sphere; source = the
    target moved by a bounded motion plus isotropic noise noise * diag."""
    Q, Qn = bumpy_sphere(rng, n)
    diag = bbox_diag(Q)
    R, t = random_motion(rng, max_angle, 0.1 * diag)
    P = _apply(R, t, Q) + rng.normal(scale=noise * diag, size=Q.shape)
    return _pack(P, Q, Qn, _gt(R, t), diag, nu_min=1e-3 * diag)


def partial_sphere_pair(rng, m=100_000, n=100_000, outliers=0.10, noise=2e-3,
                        max_angle=45.0, cap=7.0 / 13.0):
    """Target: n directions with u_z >= -cap; source: m independent samples with
    u_z <= cap (overlap measured on the source: 2 cap / (1 + cap) = 0.70 for
    cap = 7/13), a fraction of it replaced by uniform outliers in its bbox."""
    Q, Qn = bumpy_sphere(rng, n, zmin=-cap, zmax=1.0)
    diag = bbox_diag(Q)
    S, _ = bumpy_sphere(rng, m, zmin=-1.0, zmax=cap)
    R, t = random_motion(rng, max_angle, 0.1 * diag)
    S = S + rng.normal(scale=noise * diag, size=S.shape)
    S = _replace_outliers(rng, S, outliers)
    P = _apply(R, t, S)
    return _pack(P, Q, Qn, _gt(R, t), diag, nu_min=1e-3 * diag)


def resampled_sphere_pair(rng, m, n, noise=1e-3, max_angle=30.0):
    """Full-overlap pair with independent samples on both sides."""
    Q, Qn = bumpy_sphere(rng, n)
    diag = bbox_diag(Q)
    S, _ = bumpy_sphere(rng, m)
    R, t = random_motion(rng, max_angle, 0.1 * diag)
    P = _apply(R, t, S + rng.normal(scale=noise * diag, size=S.shape))
    return _pack(P, Q, Qn, _gt(R, t), diag, nu_min=1e-3 * diag)


def height_field_pair(rng, m=200_000, n=500_000, outliers=0.05, noise=1e-3,
                      max_angle=10.0, trans_frac=0.05):
    """Target: n points on [-1,1]^2 of a seeded 8-term height field with analytic
    unit normals; source: m points with x in [-0.2, 1.8] (60% overlap), uniform
    outliers, absolute noise sigma = noise."""
    hf = HeightField(rng)
    Q, Qn = hf.sample(rng, n)
    diag = bbox_diag(Q)
    S, _ = hf.sample(rng, m, xr=(-0.2, 1.8))
    S = S + rng.normal(scale=noise, size=S.shape)
    S = _replace_outliers(rng, S, outliers)
    R, t = random_motion(rng, max_angle, trans_frac * diag)
    P = _apply(R, t, S)
    return _pack(P, Q, Qn, _gt(R, t), diag, nu_min=1e-3)


def log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_pair(i, lo=2000, hi=200_000, seed_config=4):
    """Pair i of an uneven batch: M, N log-uniform in [lo, hi]; generator (full
    resample vs. partial overlap) and mode (point-to-point vs. point-to-plane)
    by independent seeded coins."""
    rng = rng_for(seed_config, i)
    m = log_uniform_int(rng, lo, hi)
    n = log_uniform_int(rng, lo, hi)
    partial = rng.uniform() < 0.5
    plane = rng.uniform() < 0.5
    if partial:
        d = partial_sphere_pair(rng, m=m, n=n)
    else:
        d = resampled_sphere_pair(rng, m=m, n=n)
    d["mode"] = 2 if plane else 1
    return d


def batch_pairs(count=256, lo=2000, hi=200_000, seed_config=4):
    """The first `count` pairs of an uneven batch (batch_pair)."""
    return [batch_pair(i, lo, hi, seed_config) for i in range(count)]


def served_request(i, lo=1000, hi=1_000_000, seed_config=5):
    """Height-field request i with M, N log-uniform in [lo, hi]."""
    rng = rng_for(seed_config, i)
    m = log_uniform_int(rng, lo, hi)
    n = log_uniform_int(rng, lo, hi)
    d = height_field_pair(rng, m=m, n=n)
    d["mode"] = 2
    return d


def served_requests(count, lo=1000, hi=1_000_000, seed_config=5, start=0):
    """Height-field requests start .. start + count - 1 (served_request)."""
    return [served_request(i, lo, hi, seed_config) for i in range(start, start + count)]
