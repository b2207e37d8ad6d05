"""Helpers shared by the GPU tests: device copies and the parity metrics."""
import numpy as np


def dev_state(st, device="cuda:0"):
    import torch
    Y = torch.tensor(st.Y, dtype=torch.float64, device=device)
    T = torch.tensor(st.T, dtype=torch.float64, device=device)
    p = torch.tensor(st.p, dtype=torch.float64, device=device)
    return Y, T, p


def gpu_integrate(mech_handle, st, dt, rtol, atol, S=None):
    """Runs the HIP integrator on a copy of st; returns host (Y, T, acc, rej, status)."""
    import torch
    Y, T, p = dev_state(st)
    Sd = None if S is None else torch.tensor(S, dtype=torch.float64, device="cuda:0")
    mech_handle.integrate(Y, T, p, dt, rtol, atol, S=Sd)
    n = st.n_cells
    acc = torch.zeros(n, dtype=torch.int32)
    rej = torch.zeros(n, dtype=torch.int32)
    sta = torch.zeros(n, dtype=torch.int32)
    mech_handle.cell_stats(acc, rej, sta)
    torch.cuda.synchronize()
    return Y.cpu().numpy(), T.cpu().numpy(), acc.numpy(), rej.numpy(), sta.numpy()


def parity(gpu, orc, floor=1e-14):
    """Relative error on graded entries: species with max(|Y_or|, |Y_gpu|) >= floor and
    T, restricted to cells whose accepted/rejected counts match the oracle's."""
    Yg, Tg, ag, rg, sg = gpu
    Yo, To, ao, ro, so = orc
    match = (ag == ao) & (rg == ro)
    graded = (np.maximum(np.abs(Yo), np.abs(Yg)) >= floor) & match[None, :]
    relY = np.abs(Yg - Yo)[graded] / np.abs(Yo)[graded] if graded.any() else np.zeros(1)
    relT = np.abs(Tg - To)[match] / np.abs(To)[match] if match.any() else np.zeros(1)
    return dict(match_frac=float(match.mean()), n_mismatch=int((~match).sum()),
                max_rel_Y=float(relY.max()), max_rel_T=float(relT.max()),
                max_rel=float(max(relY.max(), relT.max())))


def parity_all(gpu, orc, floor=1e-14):
    """Relative error over all cells (no count matching)."""
    Yg, Tg = gpu[0], gpu[1]
    Yo, To = orc[0], orc[1]
    graded = np.maximum(np.abs(Yo), np.abs(Yg)) >= floor
    relY = np.abs(Yg - Yo)[graded] / np.abs(Yo)[graded]
    relT = np.abs(Tg - To) / np.abs(To)
    return dict(max_rel_Y=float(relY.max()), max_rel_T=float(relT.max()),
                p99_rel_Y=float(np.percentile(relY, 99)))


def normalized(a, b, rtol, atol):
    """Per-entry |a - b| / (atol + rtol |b|) over Y and T; returns (max, p99 per cell)."""
    eY = np.abs(a[0] - b[0]) / (atol + rtol * np.abs(b[0]))
    eT = np.abs(a[1] - b[1]) / (atol + rtol * np.abs(b[1]))
    per_cell = np.maximum(eY.max(axis=0), eT)
    return float(per_cell.max()), float(np.percentile(per_cell, 99))


def relative(gpu, orc, floor=1e-14):
    """Largest relative error over Y (entries with max(|Y_orc|, |Y_gpu|) >= floor) and T,
    on every cell (the tolerance metric of the FP64 and mixed bars)."""
    Yg, Tg = gpu[0], gpu[1]
    Yo, To = orc[0], orc[1]
    graded = np.maximum(np.abs(Yo), np.abs(Yg)) >= floor
    relY = np.abs(Yg - Yo)[graded] / np.abs(Yo)[graded] if graded.any() else np.zeros(1)
    return float(max(relY.max(), (np.abs(Tg - To) / np.abs(To)).max()))


def envelope(orc, w, st, dt, rtol, atol, perturb=0, **kw):
    """Oracle result and the rounding envelope: how far the FMA-contracted build of the
    same oracle lands from it (normalized max / p99, relative max, count-match fraction).
    With perturb = k, k more oracle runs from inputs moved by one ulp (mass fractions
    scaled by 1 +- 2^-52, random signs) widen the normalized and relative envelope: the
    spread that rounding anywhere along the computation can produce on ill-conditioned
    steps, which the one twin build may underestimate."""
    a = orc.integrate(w.mech, st.Y, st.T, st.p, dt, rtol, atol, w.M, **kw)
    b = orc.integrate(w.mech, st.Y, st.T, st.p, dt, rtol, atol, w.M, fma=True, **kw)
    mx, p99 = normalized(b, a, rtol, atol)
    rel = relative(b, a)
    match = float(np.mean((a[2] == b[2]) & (a[3] == b[3])))
    rng = np.random.default_rng(20261)
    for _ in range(perturb):
        Yp = st.Y * (1.0 + 2.0**-52 * rng.choice([-1.0, 1.0], st.Y.shape))
        c = orc.integrate(w.mech, Yp, st.T, st.p, dt, rtol, atol, w.M, **kw)
        same = (a[2] == c[2]) & (a[3] == c[3])
        sub = lambda r: (r[0][:, same], r[1][same])
        if same.any():
            mx = max(mx, normalized(sub(c), sub(a), rtol, atol)[0])
            rel = max(rel, relative(sub(c), sub(a)))
    return a, dict(env_max=mx, env_p99=p99, env_rel=rel, env_match=match)
