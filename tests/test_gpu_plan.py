"""Batch plans (set-up once, launch many times; HIP-graph replay; concurrent
launch chains; autotuned chain count) against the one-shot batch call and the
oracle.  Every launch must be bit-identical to agn_lc_generate_batch on the
same inputs, and each graph replay must read the inputs as they are at replay
time."""
import numpy as np
import pytest

import oracle
from paper_1909_06374_amd import synth

from test_gpu_parity import agn, delta_close, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# LDS-path lengths, multi-pass lengths, and a repeated length
NS = [1024, 2**15, 3 * 2**9, 2**14, 3 * 2**13, 1024, 2**16, 6]


def _batch(prec, seed=40):
    m = agn()
    ns = list(NS)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    a_low, a_high, f_b = synth.curve_params(len(ns), seed)
    params = [m.psd_params(0.0, f_b[c], a_low[c], a_high[c]) for c in range(len(ns))]
    iters = [3 + (c % 4) for c in range(len(ns))]
    erdf = np.concatenate([synth.erdf_draw(n, seed=seed, curve_id=c) for c, n in enumerate(ns)])
    return dict(ns=ns, offs=offs, params=params, dt=[1.0] * len(ns), iters=iters,
                seeds=[seed + c for c in range(len(ns))], ids=list(range(len(ns))), erdf=erdf, prec=prec)


def _buffers(b):
    m = agn()
    nc, tot, mx = len(b["ns"]), int(np.sum(b["ns"])), max(b["iters"])
    return dict(x=torch.full((tot,), float("nan"), dtype=torch.float64, device="cuda:0"),
                d=torch.full((nc * mx,), -1.0, dtype=torch.float64, device="cuda:0"),
                done=torch.full((nc,), -7, dtype=torch.int32, device="cuda:0"),
                ws=torch.empty(m.agn_batch_workspace_size(b["ns"], b["prec"]), dtype=torch.uint8, device="cuda:0"))


def _one_shot(ctx, b, erdf_t):
    m = agn()
    o = _buffers(b)
    m.agn_lc_generate_batch(ctx, b["ns"], b["offs"], b["params"], b["dt"], b["iters"], b["seeds"], b["ids"],
                            erdf_t, -1.0, b["prec"], o["x"], o["d"], o["done"], o["ws"])
    return host(o["x"]), host(o["d"]), host(o["done"])


def _plan(ctx, b, erdf_t, o, flags, branches):
    m = agn()
    return m.agn_batch_plan_create(ctx, b["ns"], b["offs"], b["params"], b["dt"], b["iters"], b["seeds"],
                                   b["ids"], erdf_t, -1.0, b["prec"], o["x"], o["d"], o["done"],
                                   flags=flags, branches=branches, ws=o["ws"])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("flags,branches", [(0, 1), (0, 3), (1, 1), (1, 4), (4, 1), (5, 2), (8, 1), (9, 2)])
def test_plan_launch_equals_batch(gpu_ctx, prec, flags, branches):
    """Also with the 16384-key sort tile (flag 4): in FP32 it applies to the
    2^15 and 2^16 curves of the batch, whose sorts must stay exact; and with
    16 butterflies per FFT workgroup (flag 8), which must not change a bit."""
    m = agn()
    b = _batch(prec)
    erdf_t = dev(b["erdf"])
    xr, dr, doner = _one_shot(gpu_ctx, b, erdf_t)
    o = _buffers(b)
    plan = _plan(gpu_ctx, b, erdf_t, o, flags, branches)
    info = plan.info()
    # launch groups: one per length, except that in FP32 the LDS-resident
    # lengths 1024, 1536 and 2^14 (whole waves per curve) share one pack
    # launch; in FP64 only 1024 qualifies (1536 does not fit a workgroup's
    # worth of curves), and one length alone is not packed
    groups = len(set(NS)) - (2 if prec == 1 else 0)
    assert info["groups"] == groups and info["graph"] == bool(flags & m.AGN_PLAN_GRAPH)
    assert info["branches"] == max(branches, 1)
    # requested tile: 16384, or 0 (chosen by length: the lengths here, all
    # below 2^20, take 8192)
    assert info["sort_tile"] == (16384 if flags & m.AGN_PLAN_LARGE_SORT_TILE else 0)
    assert info["fft_cols"] == (16 if flags & m.AGN_PLAN_NARROW_FFT else 64)
    for rep in range(3):
        o["x"].fill_(float("nan"))
        o["done"].fill_(-7)
        m.agn_batch_plan_launch(plan)
        assert np.array_equal(host(o["x"]), xr), rep
        assert np.array_equal(host(o["d"]), dr) and np.array_equal(host(o["done"]), doner)
        # eager work between replays
        torch.cuda.synchronize()
        _ = (o["x"] * 2).sum().item()
    plan.close()


def test_graph_replay_reads_current_inputs(gpu_ctx):
    """Changing the PDF draw in place between replays changes the result to
    that of the new draw (the graph holds pointers, not values)."""
    m = agn()
    b = _batch(0, seed=41)
    erdf_t = dev(b["erdf"])
    o = _buffers(b)
    plan = _plan(gpu_ctx, b, erdf_t, o, m.AGN_PLAN_GRAPH, 2)
    m.agn_batch_plan_launch(plan)
    first = host(o["x"]).copy()
    b2 = _batch(0, seed=42)
    erdf_t.copy_(dev(b2["erdf"]))
    m.agn_batch_plan_launch(plan)
    second = host(o["x"])
    b2x = dict(b, erdf=b2["erdf"])
    xr, dr, _ = _one_shot(gpu_ctx, b2x, dev(b2["erdf"]))
    assert np.array_equal(second, xr) and not np.array_equal(first, second)
    # and against the oracle, curve by curve
    for c, n in enumerate(b["ns"]):
        p = b["params"][c]
        lo = int(b["offs"][c])
        xo, do, _, _ = oracle.generate(oracle.psd_params(p.norm, p.f_br, p.a_low, p.a_high),
                                       b2["erdf"][lo:lo + n], 1.0, b["iters"][c], b["seeds"][c], c)
        assert np.array_equal(second[lo:lo + n], xo), n
        assert delta_close(host(o["d"]).reshape(len(NS), -1)[c, :b["iters"][c]], do)
    plan.close()


def test_autotune_choice_is_cached_and_exact(gpu_ctx):
    m = agn()
    b = _batch(1, seed=43)
    erdf_t = dev(b["erdf"])
    xr, dr, doner = _one_shot(gpu_ctx, b, erdf_t)
    o = _buffers(b)
    plan = _plan(gpu_ctx, b, erdf_t, o, m.AGN_PLAN_AUTOTUNE | m.AGN_PLAN_GRAPH, 0)
    chosen = plan.info()["branches"]
    tile = plan.info()["sort_tile"]
    assert chosen in (1, 2, 4) and tile in (8192, 16384)
    m.agn_batch_plan_launch(plan)
    assert np.array_equal(host(o["x"]), xr) and np.array_equal(host(o["d"]), dr)
    assert np.array_equal(host(o["done"]), doner)
    plan2 = _plan(gpu_ctx, b, erdf_t, o, m.AGN_PLAN_AUTOTUNE, 0)
    assert plan2.info()["branches"] == chosen and plan2.info()["sort_tile"] == tile
    m.agn_batch_plan_launch(plan2)
    assert np.array_equal(host(o["x"]), xr)
    plan.close()
    plan2.close()


def test_plan_argument_errors(gpu_ctx):
    m = agn()
    b = _batch(0)
    erdf_t = dev(b["erdf"])
    o = _buffers(b)
    with pytest.raises(m.AgnError):  # unknown flag
        _plan(gpu_ctx, b, erdf_t, o, 16, 1)
    with pytest.raises(m.AgnError):  # a fixed tile and tuning exclude each other
        _plan(gpu_ctx, b, erdf_t, o, m.AGN_PLAN_AUTOTUNE | m.AGN_PLAN_LARGE_SORT_TILE, 1)
    with pytest.raises(m.AgnError):  # so do a fixed FFT width and tuning
        _plan(gpu_ctx, b, erdf_t, o, m.AGN_PLAN_AUTOTUNE | m.AGN_PLAN_NARROW_FFT, 1)
    with pytest.raises(m.AgnError):
        _plan(gpu_ctx, b, erdf_t, o, 0, 9)
    small = dict(o, ws=o["ws"][:1024])
    with pytest.raises(m.AgnError):
        _plan(gpu_ctx, b, erdf_t, small, 0, 1)
