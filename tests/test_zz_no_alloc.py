"""ace_apply_noalloc (the apply with the library's static scratch) against
ace_apply (scratch in the caller's workspace) and the FP64 oracle's apply,
through the C-ABI: two calls in a row, the second on a smaller plan and fewer
vectors, then the first again; plus the host-side size and argument checks."""
import ctypes

import numpy as np
import pytest

from oracle import ace_oracle as O
from paper_2110_07670_amd import synth

TOL = 1e-10

# (n, orbitals, vectors, seed): the second case is smaller in every size
CASES = [(48, 40, 24, 501), (32, 12, 5, 502)]


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _case(lib, n, k, nv, seed):
    import torch
    L = 0.2 * n + 3.0
    plan = lib.Plan(n, (L, L, L), k, "fp64", 0.25)
    xi = torch.from_numpy(synth.random_field((k, n, n, n), seed)).to("cuda:0")
    psi = torch.from_numpy(synth.random_field((nv, n, n, n), seed + 1)).to("cuda:0")
    return plan, xi, psi, (L ** 3) / n ** 3


def _check(lib, n, k, nv, seed):
    import torch
    plan, xi, psi, dV = _case(lib, n, k, nv, seed)
    out = torch.full_like(psi, float("nan"))
    lib.apply_noalloc_into(plan, xi, psi, out)
    ref = lib.ace_apply(plan, xi, psi)
    torch.cuda.synchronize()
    got, want = out.cpu().numpy(), ref.cpu().numpy()
    oracle = O.ace_apply(xi.cpu().numpy(), psi.cpu().numpy(), dV)
    for r in (want, oracle):
        assert O.rel_err(got, r) < TOL
        assert np.abs(got - r).max() < TOL * np.abs(r).max()
    return got


@pytest.mark.gpu
def test_apply_noalloc_matches_apply_twice_then_smaller():
    import torch
    from paper_2110_07670_amd import _lib
    assert torch.cuda.is_available()
    _say("apply_noalloc n=48 orbitals=40 vectors=24")
    first = _check(_lib, *CASES[0])
    _say("apply_noalloc n=32 orbitals=12 vectors=5")
    _check(_lib, *CASES[1])
    _say("apply_noalloc n=48 orbitals=40 vectors=24 again")
    again = _check(_lib, *CASES[0])
    assert np.array_equal(first, again)


def test_apply_noalloc_host_checks():
    from paper_2110_07670_amd import _lib
    lib = _lib.load()
    plan = _lib.Plan(32, (9.0, 9.0, 9.0), 512, "fp64", 0.25)
    fake = ctypes.c_void_p(1 << 40)
    other = ctypes.c_void_p(1 << 41)
    far = ctypes.c_void_p(1 << 42)
    # 4096 vectors of 512 orbitals: the coefficients and one partial product
    # (16 MiB each) just fit the 32 MiB scratch; 4097 do not: refused on the host
    assert lib.ace_apply_noalloc(plan.handle, None, fake, other, 4097, far) == _lib.ACE_ERR_SIZE
    assert lib.ace_apply_noalloc(plan.handle, None, None, other, 4, far) == _lib.ACE_ERR_ARG
    assert lib.ace_apply_noalloc(plan.handle, None, fake, other, 0, far) == _lib.ACE_ERR_ARG
    # out overlapping psi
    assert lib.ace_apply_noalloc(plan.handle, None, fake, other, 4, other) == _lib.ACE_ERR_ARG
