"""cbs_apply_noalloc (the operator with staging in the library's fixed scratch array, no device
allocation) against cbs_apply, the entry point whose kernels it shares: equal outputs, on two
calls in a row with the second smaller than the first (the array keeps the first call's
contents), in complex128 and complex64, on the tiny cell and the 48x48x32 workload with
projectors; and against the oracle's sparse operator on the tiny cell.  A call beyond the
array's size is refused before the device is touched."""
import numpy as np
import pytest

import workloads as W
from oracle import ham

pytestmark = pytest.mark.gpu


def _vectors(n, k, seed, dtype):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))).astype(dtype)
    z = np.exp(1j * rng.uniform(0, 2 * np.pi, k)) * rng.uniform(0.5, 2.0, k)
    return x, z


@pytest.mark.parametrize("which", ["tiny", "cfg2"])
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_noalloc_matches_apply_on_two_calls(cuda, which, dtype):
    import torch
    import paper_1709_09347_amd as cbs
    sysw = W.tiny(with_proj=True, fd_order=8) if which == "tiny" else W.config(2).systems[0]
    s = cbs.System.from_workload(sysw)
    E = 0.37
    sizes = (5, 2) if which == "tiny" else ((9, 3) if dtype == np.complex128 else (7, 2))
    for call, k in enumerate(sizes):
        xh, z = _vectors(sysw.n, k, 100 + call, dtype)
        x = torch.from_numpy(xh).to(cuda)
        want = s.apply(E, z, x)
        y = torch.full_like(x, float("nan"))
        s.apply_noalloc(E, z, x, y)
        torch.cuda.synchronize()
        print(f"{which} {np.dtype(dtype).name} call {call}: {k} vectors", flush=True)
        assert torch.equal(y, want), (call, (y - want).abs().max().item())
        if which == "tiny" and dtype == np.complex128:
            H = ham.build(sysw)
            yh = y.cpu().numpy()
            for v in range(k):
                ref = H.apply(z[v], xh[v], E)
                assert np.linalg.norm(yh[v] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_noalloc_refuses_calls_beyond_the_array(cuda):
    import torch
    import paper_1709_09347_amd as cbs
    sysw = W.config(2).systems[0]
    s = cbs.System.from_workload(sysw)
    k = 30   # 15 pairs x 2 buffers x 73,728 points x 32 B = 70.8 MB > 64 MiB
    x = torch.zeros((k, sysw.n), dtype=torch.complex128, device=cuda)
    y = torch.empty_like(x)
    with pytest.raises(cbs.CbsError) as e:
        s.apply_noalloc(0.2, np.ones(k), x, y)
    assert e.value.code == cbs.CBS_EINVAL and "scratch" in str(e.value)
