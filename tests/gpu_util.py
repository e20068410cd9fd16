"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def csr_equal(a, b):
    return np.array_equal(np.asarray(a[0]), np.asarray(b[0])) and \
        np.array_equal(np.asarray(a[1]), np.asarray(b[1]))


def gpu_list(sys, x, sig):
    """Builds on the GPU (growing the width as needed) and exports canonical CSR."""
    sys, ws = H.build_with_width(sys, dev(x), dev(sig))
    rp, cols = H.hdmd_nlist_export(sys, ws)
    return (rp.cpu().numpy(), cols.cpu().numpy().astype(np.int32)), sys, ws


def partnered(d, n, L, seed, rl, sig_a=1.0, sig_b=1.4):
    """Uniform atoms, every second one placed 0.5..1.1 rl from the previous."""
    x = inputs.uniform_positions(n, d, L, seed)
    g = np.random.default_rng(seed + 7)
    u = g.normal(size=(n // 2, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    y = x[0::2][: n // 2] + u * g.uniform(0.5, 1.1, (n // 2, 1)) * rl
    y = np.where(y >= 0.5 * L, y - L, y)
    y = np.where(y < -0.5 * L, y + L, y)
    y = np.where(y >= 0.5 * L, -0.5 * L, y)
    x[1::2][: n // 2] = y
    sig = inputs.bidisperse(n, sig_a, sig_b, seed + 1) if sig_a != sig_b else np.full(n, sig_a)
    return x, sig


def force_err(Fg, Fo):
    """max_i |F_i^gpu - F_i^oracle| / F_rms (F_rms over the oracle forces)."""
    frms = np.sqrt((Fo * Fo).sum() / len(Fo))
    return np.sqrt(((Fg - Fo) ** 2).sum(axis=1)).max() / frms
