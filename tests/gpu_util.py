"""Helpers for the GPU tests: move seeded inputs to the device and run the C ABI."""
import numpy as np
import torch


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_residual(P, ints, t1, t2):
    o, v = t1.shape
    dt1, dt2 = dev(t1), dev(t2)
    r1 = torch.empty((o, v), dtype=torch.float64, device="cuda")
    r2 = torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
    e = torch.empty((1,), dtype=torch.float64, device="cuda")
    P.ascc_residual(ints, dt1, dt2, r1, r2, e)
    torch.cuda.synchronize()
    return host(r1), host(r2), float(host(e)[0])
