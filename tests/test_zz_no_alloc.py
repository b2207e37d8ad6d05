"""The allocation-free entry point rok4e_integrate_static, through the C ABI: its results
and per-cell counts equal those of rok4e_integrate on the same inputs, bit for bit (the
same kernels; only the scratch memory differs), on two calls in a row, the second with a
smaller batch than the first; also inside a captured HIP graph replayed several times.
Batches beyond the static scratch are refused on the host."""
import numpy as np
import pytest

from gpu_util import dev_state
from paper_1712_00953_amd import synth

pytestmark = pytest.mark.gpu

A_SCALE = 1e-8


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    from paper_1712_00953_amd import rok4e as R
    R.load()
    return R


def _counts(n):
    import torch
    return [torch.full((n,), -9, dtype=torch.int32, device="cuda:0") for _ in range(3)]


def _eager(R, m, st, w):
    """rok4e_integrate on a copy of the batch; returns the state and the per-cell counts."""
    import torch
    Y, T, p = dev_state(st)
    m.integrate(Y, T, p, w.dt, w.rtol, w.atol)
    n = st.n_cells
    c = [torch.zeros(n, dtype=torch.int32) for _ in range(3)]
    m.cell_stats(*c)
    torch.cuda.synchronize()
    return Y, T, c


def _static(R, m, st, w):
    import torch
    Y, T, p = dev_state(st)
    c = _counts(st.n_cells)
    m.integrate_static(Y, T, p, w.dt, w.rtol, w.atol, *c)
    torch.cuda.synchronize()
    return Y, T, [x.cpu() for x in c]


def _same(a, b, what):
    import torch
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), what
    for x, y in zip(a[2], b[2]):
        assert torch.equal(x.cpu(), y.cpu()), what


def test_static_entry_matches_integrate_on_two_calls(R):
    # first call: the 65,536-cell flame slice (enough cells per segment in flight for the
    # hottest-first queue order, whose bins and order live in the static scratch too);
    # second call: 3,000 cells of the bimodal batch (array order), after the first call
    # left its counter, bins and order in the scratch
    for cfg, n in ((2, None), (3, 3000)):
        w = synth.workload(cfg, a_scale=A_SCALE, n_cells=n)
        st = w.states
        m = R.Mech(w.mech, M=w.M, max_attempts=20000)
        print(f"\n[static] workload {w.name} {st.n_cells} cells", flush=True)
        a = _static(R, m, st, w)
        b = _eager(R, m, st, w)
        _same(a, b, f"cfg {cfg}")
        assert np.all(a[2][2].numpy() == 0)
        m.close()


def test_static_entry_in_a_graph(R):
    import torch
    w = synth.workload(2, a_scale=A_SCALE, n_cells=32768)
    st = w.states
    m = R.Mech(w.mech, M=w.M, max_attempts=20000)
    ref = _eager(R, m, st, w)
    Y0, T0, p = dev_state(st)
    Y, T = Y0.clone(), T0.clone()
    c = _counts(st.n_cells)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            m.integrate_static(Y, T, p, w.dt, w.rtol, w.atol, *c)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        Y.copy_(Y0)
        T.copy_(T0)
        for x in c:
            x.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _same((Y, T, c), ref, f"replay {rep}")
    m.close()


def test_static_entry_refuses_oversized_batches(R):
    import ctypes as C
    import torch
    w = synth.workload(1, a_scale=A_SCALE, n_cells=8)
    m = R.Mech(w.mech, M=w.M)
    Y, T, p = dev_state(w.states)
    c = _counts(8)
    lib = R.load()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    # the host check refuses the size before anything is launched or read
    rc = lib.rok4e_integrate_static(R.STATIC_MAX_CELLS + 1, m.handle, ptr(Y), ptr(T), ptr(p), None,
                                    w.dt, w.rtol, w.atol, ptr(c[0]), ptr(c[1]), ptr(c[2]), None)
    assert rc == R.ESTATIC
    assert "static scratch" in R.strerror(rc)
    with pytest.raises(ValueError):
        m.integrate_static(Y, T, p, w.dt, w.rtol, w.atol, c[0], c[1], None)
    m.integrate_static(Y[:, :0], T[:0], p[:0], w.dt, w.rtol, w.atol, c[0][:0], c[1][:0], c[2][:0], n_cells=0)
    torch.cuda.synchronize()
    m.close()
