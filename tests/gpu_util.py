"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import torch

import paper_1405_7487_amd as F


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_fmm(x, q, p, theta, ncrit, precision, dtype=torch.float64):
    plan = F.Plan(dev(x, dtype), F.Params(p=p, theta=theta, ncrit=ncrit, precision=precision))
    phi, E = plan.evaluate(dev(q, dtype))
    torch.cuda.synchronize()
    return plan, host(phi), host(E)
