"""Helpers shared by the GPU tests: seeded frames to device tensors, oracle runs
on the same float32-rounded inputs, and the error metrics of the parity bar."""
import numpy as np
import torch

from oracle import pme as opme

E_REL_TOL = 1e-5      # relative energy error (E_recip and E^lr)
RMS_REL_TOL = 1e-4    # ||a - b||_rms / ||b||_rms for gradients and HVP outputs


def dev():
    return torch.device("cuda", 0)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def to_dev(frame, with_q=True, with_mu=True):
    d = dev()
    pos = torch.tensor(frame.pos, dtype=torch.float32, device=d)
    q = torch.tensor(frame.q, dtype=torch.float32, device=d) if with_q else None
    mu = torch.tensor(frame.mu, dtype=torch.float32, device=d) if with_mu else None
    box = torch.tensor(np.asarray(frame.box, dtype=np.float64), device=d)
    return pos, q, mu, box


def oracle_forward(frame, mesh, p, alpha, gamma=1.0, prefactor=1.0, with_q=True, with_mu=True):
    return opme.forward(f32(frame.pos), f32(frame.q) if with_q else None,
                        f32(frame.mu) if with_mu else None, frame.box, mesh, p, alpha,
                        gamma=gamma, prefactor=prefactor)


def oracle_hvp(frame, mesh, p, alpha, v, gamma=1.0, prefactor=1.0):
    return opme.hvp(f32(frame.pos), f32(frame.q), f32(frame.mu), frame.box, mesh, p, alpha,
                    v_pos=f32(v[0]), v_q=f32(v[1]), v_mu=f32(v[2]), gamma=gamma,
                    prefactor=prefactor)


def rms_rel(a, b, floor=0.0):
    """||a - b||_rms / max(||b||_rms, floor); floor is a physical scale for cases
    whose exact value vanishes (e.g. the mesh self-force on a lone atom)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.sqrt(np.mean(b * b))), floor)
    return float(np.sqrt(np.mean((a - b) ** 2)) / (den if den > 0 else 1.0))


def rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def host(t):
    return t.detach().double().cpu().numpy()
