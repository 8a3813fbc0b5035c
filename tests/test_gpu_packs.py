"""The persistent launch of LDS-resident curves (packs): a batch with several
LDS-resident lengths runs every such curve in one k_lds_packs launch, several
curves of one length sharing a workgroup.  Each curve's arithmetic is the
same as in its own launch, so the results must be bit-identical to one
agn_lc_generate call per curve -- with different iteration counts per curve,
the stopping rule ending curves of one pack at different iterations, partly
filled packs, and an invalid draw in one curve -- and, in FP64, to the
oracle."""
import numpy as np
import pytest

import oracle
from paper_1909_06374_amd import synth

from test_gpu_parity import agn, delta_close, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def lengths(prec):
    # every LDS-resident length class with whole waves per curve; counts leave
    # the last pack of each length part-filled
    out = []
    for n, k in [(1024, 11), (1536, 3), (2048, 5), (3072, 2), (4096, 3), (6144, 2), (8192, 2), (12288, 2)]:
        out += [n] * k
    if prec == 1:
        out += [16384] * 2
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tol", [-1.0, 0.05])
def test_packs_equal_single_calls(gpu_ctx, prec, tol):
    m = agn()
    ns = lengths(prec)
    nc = len(ns)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    a_low, a_high, f_b = synth.curve_params(nc, 9)
    params = [m.psd_params(0.0, f_b[c], a_low[c], a_high[c]) for c in range(nc)]
    iters = [4 + (7 * c) % 9 for c in range(nc)]
    seeds = [700 + c for c in range(nc)]
    erdf = np.concatenate([synth.erdf_draw(n, seed=91, curve_id=c) for c, n in enumerate(ns)])
    bad = 5  # one invalid draw (a zero) in a curve of the first length
    erdf[offs[bad] + 17] = 0.0
    et = dev(erdf)
    mx = max(iters)
    x = torch.full((int(np.sum(ns)),), float("nan"), dtype=torch.float64, device="cuda:0")
    d = torch.full((nc * mx,), -1.0, dtype=torch.float64, device="cuda:0")
    done = torch.full((nc,), -7, dtype=torch.int32, device="cuda:0")
    ws = torch.empty(m.agn_batch_workspace_size(ns, prec), dtype=torch.uint8, device="cuda:0")
    gpu_ctx.kernel_times(reset=True)
    gpu_ctx.set_profiling(True)
    m.agn_lc_generate_batch(gpu_ctx, ns, offs, params, [1.0] * nc, iters, seeds, list(range(nc)), et, tol, prec,
                            x, d, done, ws)
    torch.cuda.synchronize()
    gpu_ctx.set_profiling(False)
    kt = gpu_ctx.kernel_times(reset=True)
    # one persistent launch; in FP64 the 3 * 2^k lengths 1536 and 3072 do not
    # fit a workgroup's worth of curves in the LDS and keep their own launches
    assert kt["lds_packs"][1] == 1 and kt["lds_iterate"][1] == (0 if prec == 1 else 2), kt
    xb, db, doneb = host(x), host(d).reshape(nc, mx), host(done)
    for c, n in enumerate(ns):
        ws1 = torch.empty(m.agn_workspace_size(n, prec), dtype=torch.uint8, device="cuda:0")
        x1 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        d1 = torch.full((iters[c],), -1.0, dtype=torch.float64, device="cuda:0")
        done1 = torch.full((1,), -7, dtype=torch.int32, device="cuda:0")
        m.agn_lc_generate(gpu_ctx, params[c], et[offs[c]:offs[c] + n], n, 1.0, iters[c], tol, seeds[c], c, prec, x1,
                          d1, done1, ws1)
        k = int(host(done1)[0])
        assert doneb[c] == k, (c, n, doneb[c], k)
        if c == bad:
            assert k == -1
            continue
        assert np.array_equal(xb[offs[c]:offs[c] + n], host(x1)), (c, n)
        assert np.array_equal(db[c, :iters[c]], host(d1)), (c, n)
        if prec == 0 and c % 4 == 0:
            p = params[c]
            xr, dr, doner, _ = oracle.generate(oracle.psd_params(p.norm, p.f_br, p.a_low, p.a_high),
                                               erdf[offs[c]:offs[c] + n], 1.0, iters[c], seeds[c], c, tol=tol)
            assert doner == k and np.array_equal(xr, host(x1)) and delta_close(host(d1)[:k], dr[:k])
    if tol > 0:
        print("iterations done per curve:", doneb.tolist())
