"""The allocation-free entry point tmamg_force_from_fields_noalloc (for
callers that cannot allocate device memory) against the allocating
tmamg_force_from_fields on the same inputs: two calls in a row through the
same static scratch array, the second on a smaller lattice, then a lattice
beyond the array's limit, which is refused."""
import pytest
import torch

from tests.gpu_common import DEV, links, spinors, kappa_of

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


def make(dims, seed):
    U, Ud = links(dims, 0.35, seed)
    s = tm.Solver(dims, tm.default_params(nlevels=0, setup_iters=0, init_smooth=0))
    s.setup(Ud, kappa_of(-0.15), 1.6, 0.01)
    return s


def test_noalloc_force_matches_allocating_entry_point():
    for dims, seed in (((8, 8, 8, 16), 7101), ((4, 4, 8, 8), 7102)):
        say("allocation-free force on", dims)
        s = make(dims, seed)
        X = spinors(dims, seed + 1, 1)[1]
        Y = spinors(dims, seed + 2, 1)[1]
        shape = (4,) + tuple(reversed(dims)) + (3, 3)
        F_ref = torch.empty(shape, dtype=torch.complex128, device=DEV)
        F_na = torch.full(shape, float("nan"), dtype=torch.complex128, device=DEV)
        s.force_from_fields(X, Y, F_ref)
        s.force_from_fields_noalloc(X, Y, F_na)
        torch.cuda.synchronize()
        err = float((F_na - F_ref).abs().max() / F_ref.abs().max())
        say(f"  max deviation over the largest entry {err:.2e}, identical: {torch.equal(F_na, F_ref)}")
        assert err <= 1e-14
        s.close()


def test_noalloc_force_refuses_lattices_beyond_its_scratch():
    dims = (16, 16, 16, 48)   # 196,608 sites > 134,432
    say("allocation-free force on", dims, "(beyond the limit)")
    s = make(dims, 7103)
    X = spinors(dims, 7104, 1)[1]
    F = torch.empty((4,) + tuple(reversed(dims)) + (3, 3), dtype=torch.complex128, device=DEV)
    with pytest.raises(tm.TmamgError) as e:
        s.force_from_fields_noalloc(X, X, F)
    assert e.value.status == tm.binding.EINVAL and "134432 sites" in str(e.value)
    s.close()
