"""Helpers shared by the GPU tests: run the library on a workload and compare
it with the FP64 oracle."""
import numpy as np

from oracle import expansion as ex


def rel_l2(a, b):
    """Relative L2 distance; complex inputs (spectra, their gradients) are
    compared as complex numbers, real and imaginary parts both."""
    a = np.asarray(a)
    b = np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = a.astype(dt)
    b = b.astype(dt)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def per_instance_rel(got, ref):
    return max(rel_l2(g, r) for g, r in zip(got, ref))


def plan_args(p):
    """Windows argument of Plan for a workload."""
    if p.separable:
        return (p.w_rows, p.w_cols)
    return p.w


def gpu_run(p, v=None, device="cuda"):
    """(H_m u, H_m^* v) from the library for workload ``p`` (v defaults to u)."""
    import torch
    import paper_1604_04374_amd as pcm
    print(f"[gpu] {p.name}: plan + apply + adjoint", flush=True)
    u = torch.from_numpy(p.u).to(device)
    vv = u if v is None else torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device)
    with pcm.Plan(plan_args(p), p.h, batch=p.batch) as plan:
        y = plan.apply(u)
        x = plan.apply_adjoint(vv)
        torch.cuda.synchronize()
        return y.cpu().numpy(), x.cpu().numpy()


def oracle_fft(p, v=None):
    """FP64 FFT-form oracle on the float32 inputs (validated against the direct
    sums at small sizes by the oracle's pins)."""
    w = p.dense_windows()
    h = p.h.astype(np.float64)
    u = p.u.astype(np.float64)
    vv = u if v is None else np.asarray(v, np.float64)
    return ex.apply_fft(u, w, h), ex.adjoint_fft(vv, w, h)


def oracle_direct(p, v=None):
    w = p.dense_windows()
    h = p.h.astype(np.float64)
    u = p.u.astype(np.float64)
    vv = u if v is None else np.asarray(v, np.float64)
    return ex.apply_direct(u, w, h), ex.adjoint_direct(vv, w, h)


def sampled_direct(p, y_gpu, x_gpu, n_samples=256, seed=0, v=None):
    """Max relative error of sampled outputs against the direct sums, scaled
    by the RMS of the oracle's sampled values."""
    rng = np.random.default_rng(seed)
    w = p.dense_windows()
    h = p.h.astype(np.float64)
    errs = []
    for b in range(p.u.shape[0]):
        idx = rng.choice(p.n_total, size=min(n_samples, p.n_total), replace=False)
        u = p.u[b].astype(np.float64)
        vv = u if v is None else np.asarray(v[b], np.float64)
        ry = ex.apply_direct_at(u, w, h, idx)
        rx = ex.adjoint_direct_at(vv, w, h, idx)
        gy = y_gpu[b].ravel()[idx]
        gx = x_gpu[b].ravel()[idx]
        errs.append(np.linalg.norm(gy - ry) / np.linalg.norm(ry))
        errs.append(np.linalg.norm(gx - rx) / np.linalg.norm(rx))
    return max(errs)
