"""The evaluation entry point that allocates nothing (rsph_eval_rates_noalloc),
called through the C-ABI on caller-owned device buffers, against the
allocating path (rsph_set_particles + rsph_eval_rates + rsph_read_particles):
the same kernels over the same layout, so the rates must be equal bit for bit,
in both forms, on two calls in a row (the second with fewer particles, so the
scratch array still holds the first call's larger contents)."""
import sys

import numpy as np
import pytest

from paper_2503_16082_amd import workloads as WL

pytestmark = pytest.mark.gpu

rsph = pytest.importorskip("paper_2503_16082_amd.rsph")
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def perturbed(w, seed):
    p = dict(w["params"])
    rng = np.random.default_rng(seed)
    n, d = w["pos"].shape
    vel = 0.05 * p["c0"] * rng.normal(size=(n, d))
    rho = np.asarray(p["rho0"])[w["phase"]] * (1.0 + 0.01 * rng.normal(size=n))
    return p, w["pos"], vel, w["phase"], rho


def allocating(p, pos, vel, phase, rho, precision):
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, vel, phase, rho=rho)
    s.eval_rates()
    out = s.read("acc"), s.read("rate_drho")
    s.close()
    return out


def no_alloc(p, pos, vel, phase, rho, precision):
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    dpos, dvel, drho_in = t(pos, torch.float64), t(vel, torch.float64), t(rho, torch.float64)
    dphase = t(phase, torch.int32)
    n, d = pos.shape
    acc = torch.full((n, d), float("nan"), dtype=torch.float64, device=dev)
    rate = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    rsph.eval_rates_noalloc(p, n, dpos.data_ptr(), dvel.data_ptr(), dphase.data_ptr(), acc.data_ptr(),
                            rate.data_ptr(), rho=drho_in.data_ptr(), precision=precision,
                            stream=stream.cuda_stream)
    return acc.cpu().numpy(), rate.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_equals_the_allocating_path_twice(precision, dim):
    if dim == 2:
        cases = [WL.static_droplet_2d(n_side=120, seed=1), WL.static_droplet_2d(n_side=50, seed=2)]
    else:
        cases = [WL.static_droplet_3d(n_side=30, R=0.3, seed=1), WL.static_droplet_3d(n_side=16, R=0.3, seed=2)]
    for k, w in enumerate(cases):
        p, pos, vel, phase, rho = perturbed(w, 10 + k)
        say(f"no-alloc call {k}: dim={dim} precision={precision} n={len(pos)}")
        a_ref, r_ref = allocating(p, pos, vel, phase, rho, precision)
        a, r = no_alloc(p, pos, vel, phase, rho, precision)
        assert np.isfinite(a).all() and np.isfinite(r).all()
        assert np.array_equal(a, a_ref), np.abs(a - a_ref).max()
        assert np.array_equal(r, r_ref), np.abs(r - r_ref).max()


def test_noalloc_rejects_oversized_and_invalid_input():
    w = WL.static_droplet_3d(n_side=48, R=0.3)  # 110,592 particles: beyond the 64 MiB scratch
    p = dict(w["params"])
    n = len(w["pos"])
    dev = torch.device("cuda:0")
    pos = torch.tensor(w["pos"], dtype=torch.float64, device=dev)
    vel = torch.zeros_like(pos)
    ph = torch.tensor(w["phase"], dtype=torch.int32, device=dev)
    acc = torch.empty_like(pos)
    rate = torch.empty(n, dtype=torch.float64, device=dev)
    with pytest.raises(rsph.RsphError) as e:
        rsph.eval_rates_noalloc(p, n, pos.data_ptr(), vel.data_ptr(), ph.data_ptr(), acc.data_ptr(),
                                rate.data_ptr(), precision=0)
    assert e.value.name == "EINVAL" and "scratch" in str(e.value)
    # a phase outside {0, 1, 2} is caught on the device and rejected
    w = WL.static_droplet_2d(n_side=30)
    p = dict(w["params"])
    bad = w["phase"].copy()
    bad[7] = 5
    pos = torch.tensor(w["pos"], dtype=torch.float64, device=dev)
    ph = torch.tensor(bad, dtype=torch.int32, device=dev)
    acc = torch.empty_like(pos)
    rate = torch.empty(len(bad), dtype=torch.float64, device=dev)
    with pytest.raises(rsph.RsphError) as e:
        rsph.eval_rates_noalloc(p, len(bad), pos.data_ptr(), torch.zeros_like(pos).data_ptr(), ph.data_ptr(),
                                acc.data_ptr(), rate.data_ptr(), precision=1)
    assert e.value.name == "EINVAL"
    # and a valid call afterwards still works
    a, r = no_alloc(p, w["pos"], np.zeros_like(w["pos"]), w["phase"],
                    np.asarray(p["rho0"])[w["phase"]], 1)
    a_ref, r_ref = allocating(p, w["pos"], np.zeros_like(w["pos"]), w["phase"],
                              np.asarray(p["rho0"])[w["phase"]], 1)
    assert np.array_equal(a, a_ref) and np.array_equal(r, r_ref)
