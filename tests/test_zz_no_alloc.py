"""les_diagnostics_noalloc (the entry point that allocates nothing: its
scratch is a static device array of the library) against les_diagnostics
on the same states: the same kernels in the same order, so the totals and
the azimuthal sums agree bitwise.  Two calls in a row share the GPU's
static array, the second on a smaller mesh (fewer partial sums) whose
result must not see the first call's leftovers."""
import pytest
import torch

from _helpers import announce, make_solver
from cases import problems

pytestmark = pytest.mark.gpu


def _both(s, Qn):
    from paper_2301_00817_amd import binding as B
    nx, nr, _ = s.shape
    st = torch.cuda.current_stream().cuda_stream
    out = []
    for fn in (B.les_diagnostics, B.les_diagnostics_noalloc):
        totals = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        s1 = torch.zeros((5, nr, nx), dtype=torch.float64, device="cuda")
        s2 = torch.zeros_like(s1)
        fn(s.ctx, Qn.data_ptr(), totals.data_ptr(), s1.data_ptr(), s2.data_ptr(), st)
        torch.cuda.synchronize()
        out.append((totals.cpu(), s1.cpu(), s2.cpu()))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_diagnostics_match_twice_second_smaller(precision):
    announce("noalloc diagnostics", precision)
    big = problems.jet_problem(288, 160, 64, seed=2)       # 2048 blocks of partial sums
    small = problems.jet_problem(40, 22, 16, seed=3)       # 56 blocks
    results = []
    for pb in (big, small):
        s = make_solver(pb, precision=precision)
        Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
        s.rk5_step(Qn, 1)
        ref, got = _both(s, Qn)
        for a, b in zip(ref, got):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)
        results.append(got[0])
        s.close()
    # the small mesh's totals are its own (not the large mesh's leftovers)
    assert not torch.equal(results[0], results[1])


def test_noalloc_diagnostics_totals_only():
    """totals without the statistics, and the statistics without totals."""
    from paper_2301_00817_amd import binding as B
    announce("noalloc diagnostics parts")
    pb = problems.box_problem(24)
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    st = torch.cuda.current_stream().cuda_stream
    t_ref = s.diagnostics(Qn)
    t = torch.empty(5, dtype=torch.float64, device="cuda")
    B.les_diagnostics_noalloc(s.ctx, Qn.data_ptr(), t.data_ptr(), None, None, st)
    nx, nr, _ = s.shape
    s1 = torch.zeros((5, nr, nx), dtype=torch.float64, device="cuda")
    B.les_diagnostics_noalloc(s.ctx, Qn.data_ptr(), None, s1.data_ptr(), None, st)
    s1_ref, _ = s.new_stats()
    B.les_diagnostics(s.ctx, Qn.data_ptr(), None, s1_ref.data_ptr(), None, st)
    torch.cuda.synchronize()
    assert torch.equal(t, t_ref)
    assert torch.equal(s1, s1_ref)
    with pytest.raises(B.LesError) as e:
        B.les_diagnostics_noalloc(s.ctx, None, t.data_ptr(), None, None, st)
    assert e.value.code == B.LES_EINVAL
    s.close()
