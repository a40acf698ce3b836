"""The diagonal-block entry point that allocates nothing (dg_assemble_diag_noalloc),
through the C ABI, against dg_assemble_diag (Sec. 6.3 blocks): bit for bit, on
two calls in a row, the second on a smaller mesh (the shared device scratch
keeps the first call's contents), and its refusal of a mesh whose neighbour
traces exceed the fixed scratch."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1812_04789_amd import binding, inputs          # noqa: E402

L = 2 * math.pi


def _ctx(n, p, curved):
    vtx = inputs.box_vertices(n, (0, 0, 0), (L, L, L), amp=0.1) if curved else None
    return binding.Context(n, (0, 0, 0), (L, L, L), p, vertices=vtx, gamma=1.4, mu=0.02, Pr=0.71, eta=7.0)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("first,second", [(((3, 2, 2), 3, True), ((2, 2, 1), 2, False)),
                                          (((4, 3, 3), 2, False), ((2, 2, 2), 1, True))])
def test_noalloc_diag_blocks_equal_the_allocating_entry_point(first, second):
    for k, (n, p, curved) in enumerate((first, second)):
        print("no-alloc blocks call", k, n, p, curved, flush=True)
        ctx = _ctx(n, p, curved)
        W = _dev(inputs.random_state(ctx.ne, p, seed=101 + k))
        nb = 5 * ctx.nv
        out = torch.full((ctx.ne * nb * nb,), float("nan"), dtype=torch.float64, device="cuda")
        got = ctx.assemble_diag_noalloc(W, 7.5, out)
        ref = ctx.assemble_diag(W, 7.5)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (k, n, p)
        ctx.close()


def test_noalloc_rejects_a_mesh_beyond_the_scratch():
    """33^3 elements at p = 1 need 138 MB of neighbour traces (35,937 x 480
    doubles), more than the 128 MiB scratch: refused with DG_EINVAL on the
    host, before any launch; the full-size output is left untouched."""
    n = (33, 33, 33)
    ctx = binding.Context(n, (0, 0, 0), (L, L, L), 1, gamma=1.4, mu=0.02, Pr=0.71, eta=7.0)
    assert ctx.ne * 6 * 4 * 20 * 8 > 128 * 2 ** 20
    W = _dev(inputs.random_state(ctx.ne, 1, seed=7))
    nb = 5 * ctx.nv
    out = torch.zeros(ctx.ne * nb * nb, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.DGError) as ei:
        ctx.assemble_diag_noalloc(W, 1.0, out)
    assert ei.value.status == binding.DG_EINVAL
    assert "too large" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    ctx.close()
