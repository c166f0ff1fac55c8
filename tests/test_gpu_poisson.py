"""GPU parity of the red-black SOR Poisson solver on patch groups (Sec. 2.3,
Eqs. Residual and SOR; Sec. 3.2) through the C ABI:

* with a fixed number of iterations the device and the oracle do the same
  operations in the same order: identical bits in FP64 and FP32;
* run to convergence (default omega and stopping rule) both reach the
  discrete solution: FP64 within 1e-11 and FP32 within 1e-5 of the largest
  potential, iteration counts within one;
* the exact quadratic solution is reached on the device;
* at full size (4096 groups, a 256^3 domain's worth) every group stops by
  the rule before the limit, and sampled groups match the oracle.
"""
import math

import numpy as np
import pytest
import torch

from oracle import poisson
from gpu_helpers import note
from paper_0907_3390_amd import tvd, workloads as wl

pytestmark = pytest.mark.gpu
N, M = 16, 18


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _groups(n_groups, seed, npd):
    """Seeded patch groups: lognormal densities, Dirichlet ghosts and initial
    guesses from a smooth potential plus noise; one zone size per group."""
    r = wl.rng(seed)
    rho = r.lognormal(0.0, 0.5, size=(n_groups, N, N, N))
    c = (np.arange(-1, N + 1) + 0.5) / N
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    base = np.sin(2 * x) * np.cos(3 * y) + 0.5 * z * z
    phi = base[None] * r.uniform(0.5, 2.0, size=(n_groups, 1, 1, 1))
    phi = phi + 0.01 * r.standard_normal(phi.shape)
    dh = 1.0 / (N * 2.0 ** r.integers(0, 4, size=n_groups))
    return phi.astype(npd), rho.astype(npd), dh


def _device(ctx, dtype, phi, rho, dh, grav=1.0, **kw):
    code = tvd.dtype_code(dtype)
    ng = phi.shape[0]
    out = torch.zeros(ng * N ** 3, dtype=dtype, device="cuda")
    iters = torch.zeros(ng, dtype=torch.int32, device="cuda")
    resid = torch.zeros(ng, dtype=torch.float64, device="cuda")
    ctx.tvd_poisson_sor(code, ng, torch.from_numpy(np.ascontiguousarray(phi)).cuda(),
                        torch.from_numpy(np.ascontiguousarray(rho)).cuda(), out, grav,
                        d_dh=torch.from_numpy(np.ascontiguousarray(dh, dtype=np.float64)).cuda(),
                        iters=iters, resid=resid, **kw)
    torch.cuda.synchronize()
    return (out.cpu().numpy().reshape(ng, N, N, N), iters.cpu().numpy(), resid.cpu().numpy())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("iters", [1, 7, 40])
def test_fixed_iterations_bitwise(ctx, dtype, iters):
    note(f"SOR fixed iterations dtype={dtype} iters={iters}")
    npd = np.float64 if dtype == torch.float64 else np.float32
    phi, rho, dh = _groups(24, seed=200 + iters, npd=npd)
    G, omega = 0.8, 1.7
    got, it, _ = _device(ctx, dtype, phi, rho, dh, grav=G, omega=omega, min_iter=iters,
                         max_iter=iters)
    src = poisson.source(rho, G, dh)
    want, wit, _ = poisson.sor(phi, src, omega=omega, min_iter=iters, max_iter=iters)
    assert np.all(it == iters) and np.all(wit == iters)
    assert np.array_equal(got, want[:, 1:-1, 1:-1, 1:-1])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_converged_matches_oracle(ctx, dtype):
    note(f"SOR to convergence dtype={dtype}")
    npd = np.float64 if dtype == torch.float64 else np.float32
    phi, rho, dh = _groups(16, seed=210, npd=npd)
    got, it, res = _device(ctx, dtype, phi, rho, dh, max_iter=2000)
    want, wit, wres = poisson.sor(phi, poisson.source(rho, 1.0, dh), max_iter=2000)
    scale = np.abs(want).max()
    err = np.abs(got - want[:, 1:-1, 1:-1, 1:-1]).max() / scale
    note(f"  iterations {it.min()}..{it.max()} (oracle {wit.min()}..{wit.max()}), max rel diff {err:.1e}")
    assert np.all(np.abs(it - wit) <= 1) and np.all(it < 2000)
    assert err <= (1e-11 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_quadratic_exact_on_device(ctx, dtype):
    npd = np.float64 if dtype == torch.float64 else np.float32
    h = 1.0 / N
    c = (np.arange(-1, N + 1) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    exact = 0.7 * x * x - 0.4 * y * y + 1.3 * z * z + 0.2 * x + 1.0
    G = 1.0
    rho = np.full((1, N, N, N), 2 * (0.7 - 0.4 + 1.3) / (4 * math.pi * G))
    phi0 = exact.copy()[None]
    phi0[:, 1:-1, 1:-1, 1:-1] = 0.0
    got, it, _ = _device(ctx, dtype, phi0.astype(npd), rho.astype(npd), np.array([h]), grav=G,
                         max_iter=3000)
    err = np.abs(got[0] - exact[1:-1, 1:-1, 1:-1]).max() / np.abs(exact).max()
    note(f"  quadratic {dtype}: {it[0]} iterations, max rel error {err:.1e}")
    assert err <= (1e-12 if dtype == torch.float64 else 1e-4)


def test_full_size_fp32(ctx):
    """4096 groups (the patch groups of a 256^3 domain), FP32, default omega
    and stopping rule: every group stops by the rule, sampled groups match
    the oracle's converged solution."""
    note("SOR full size, 4096 groups fp32")
    phi, rho, dh = _groups(4096, seed=220, npd=np.float32)
    got, it, res = _device(ctx, torch.float32, phi, rho, dh, max_iter=1000)
    note(f"  iterations {it.min()}..{it.max()}, mean {it.mean():.1f}")
    assert np.all(it < 1000)
    picks = wl.rng(221).choice(4096, size=24, replace=False)
    want, wit, _ = poisson.sor(phi[picks], poisson.source(rho[picks], 1.0, dh[picks]), max_iter=1000)
    err = np.abs(got[picks] - want[:, 1:-1, 1:-1, 1:-1]).max() / np.abs(want).max()
    assert np.all(np.abs(it[picks] - wit) <= 1) and err <= 1e-5
