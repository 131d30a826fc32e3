"""mu_chi2_eval_static: the allocation-free variant of mu_chi2_eval (its
partial slots live in a static per-device array).  Two calls in a row, the
second on a smaller input, each bit for bit equal to mu_chi2_eval on the same
device tensors and within a relative 1e-10 of the oracle (Eqs. 2-3); a call
needing more slots than the array holds is refused and leaves later calls
working."""

import numpy as np
import pytest

from oracle import model
from paper_1604_02334_amd import api

from _workloads import c1, c2, perturbed

pytestmark = pytest.mark.gpu
REL = 1e-10


def test_static_entry_point_matches_mu_chi2_eval():
    import torch
    print("[case] mu_chi2_eval_static: C2 x 8 vectors, then C1 x 3 vectors", flush=True)
    ctx = api.Context(0)
    try:
        cases = []
        for (cfg, counts), n_vec, seed in ((c2(), 8, 51), (c1(), 3, 52)):
            th = api.Theory(ctx, cfg["theory"])
            d = api.Data(ctx, cfg["histos"], counts)
            P = np.stack([perturbed(cfg["p_true"], 1e-3, seed + v) for v in range(n_vec)])
            cases.append((cfg, counts, th, d, P))
        with torch.cuda.stream(ctx.torch_stream):
            for cfg, counts, th, d, P in cases:
                n_vec, n_histo = P.shape[0], len(cfg["histos"])
                for kind in ("chi2", "poisson"):
                    Pd = torch.tensor(P, dtype=torch.float64, device="cuda")
                    ref, ref_h = api.chi2_eval(ctx, d, th, Pd, kind, per_histo=True)
                    out = torch.full((n_vec,), float("nan"), dtype=torch.float64, device="cuda")
                    ph = torch.full((n_vec, n_histo), float("nan"), dtype=torch.float64, device="cuda")
                    api.chi2_eval_static(ctx, d, th, Pd, out, ph, kind)
                    torch.cuda.synchronize()
                    assert torch.equal(out, ref), (kind, out, ref)
                    assert torch.equal(ph, ref_h), kind
                    got = out.cpu().numpy()
                    for v in range(n_vec):
                        o = model.cost(cfg["theory"], cfg["histos"], counts, P[v], kind)
                        assert abs(got[v] - o) <= REL * o, (kind, v, got[v], o)
            # more slots than the static array holds: refused, nothing enqueued
            cfg, counts, th, d, P = cases[0]
            ctx.tile = 64
            Pd = torch.tensor(P[:2], dtype=torch.float64, device="cuda")
            out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
            with pytest.raises(api.A.MuError) as e:
                api.chi2_eval_static(ctx, d, th, Pd, out)
            assert e.value.status == api.A.MU_E_UNSUPPORTED
            torch.cuda.synchronize()
            assert torch.all(out == -1.0)
            ctx.tile = 0
            # and the next call works
            api.chi2_eval_static(ctx, d, th, Pd, out)
            ref = api.chi2_eval(ctx, d, th, Pd)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
        for _, _, th, d, _ in cases:
            th.close()
            d.close()
    finally:
        ctx.close()
