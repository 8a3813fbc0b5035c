"""Host-side argument checks of the Python binding.

The C ABI takes plain device pointers and cannot see how large a buffer is,
so the binding checks every tensor against the extent the call will touch
(and its dtype, device and layout) and raises before anything reaches the
library.  These run on the CPU with stand-in tensor objects: each call below
fails in the binding, so no device is needed.
"""
import os
import types

import pytest

import paper_1909_06374_amd as agn


class Fake:
    """Just enough of a torch tensor for the binding's checks."""

    def __init__(self, numel, dtype="torch.float64", cuda=True, contiguous=True, index=0):
        self._numel = numel
        self.dtype = dtype
        self.is_cuda = cuda
        self._contiguous = contiguous
        self.device = types.SimpleNamespace(index=index)

    def numel(self):
        return self._numel

    def element_size(self):
        return 8

    def is_contiguous(self):
        return self._contiguous

    def data_ptr(self):
        return 0x10000


CTX = types.SimpleNamespace(device=0, handle=None)


def needs_lib():
    if not os.path.exists(agn.LIB_PATH):
        pytest.skip("libagn.so not built")


def test_buf_accepts_and_rejects():
    assert agn._buf(None) is None
    assert agn._buf(Fake(10), "x", agn._F64, 10, 0).value == 0x10000
    assert agn._buf(Fake(10, "torch.uint32"), "r", agn._I32, 3, 0).value == 0x10000
    bad = [(Fake(9), agn._F64, 10, 0, "at least 10"),
           (Fake(10, "torch.float32"), agn._F64, 10, 0, "dtype"),
           (Fake(10, cuda=False), agn._F64, 10, 0, "GPU tensor"),
           (Fake(10, contiguous=False), agn._F64, 10, 0, "contiguous"),
           (Fake(10, index=1), agn._F64, 10, 0, "cuda:1")]
    for t, dt, need, dev, msg in bad:
        with pytest.raises(agn.AgnError) as e:
            agn._buf(t, "x", dt, need, dev)
        assert e.value.code == agn.AGN_EINVAL and msg in str(e.value)


def test_extent():
    assert agn._extent([], []) == 0
    assert agn._extent([4, 8], [0, 10]) == 18
    assert agn._extent([4, 8], [20, 10], lambda k: k // 2 + 1) == 23
    assert agn._extent([4, 8], [-5, 2]) == 10  # a negative offset is the library's to reject


def test_nbins_matches_the_library():
    needs_lib()
    got = agn._nbins([1024, 2048, 1024, 1000, 2], 0.1)
    assert list(got[:3]) == [agn.agn_log_bin_count(1024, 0.1), agn.agn_log_bin_count(2048, 0.1),
                             agn.agn_log_bin_count(1024, 0.1)]
    assert list(got[3:]) == [0, 0]  # unsupported lengths: the library rejects the call
    assert list(agn._nbins([1024], 0.0)) == [0]


def calls():
    """(entry point, kwargs with exactly one buffer one element short, buffer name)."""
    psd = agn.psd_params(0.0, 1 / 200.0, 1.0, 2.0)
    n = 1024
    one = dict(params=psd, erdf=Fake(n), n=n, dt=1.0, iters=5, tol=-1.0, seed=1, curve_id=0, prec=agn.AGN_FP64,
               x_out=Fake(n), delta_out=Fake(5), iters_done=Fake(1, "torch.int32"), ws=Fake(1 << 20, "torch.uint8"))
    it = dict(amp=Fake(n // 2 + 1, "torch.float32"), x0=Fake(n), n=n, iters=5, tol=-1.0, prec=agn.AGN_FP32,
              x_out=Fake(n), delta_out=Fake(5), iters_done=Fake(1, "torch.int32"), rank_out=Fake(n, "torch.int32"),
              ws=Fake(1 << 20, "torch.uint8"))
    ns, offs = [1024, 2048], [2048, 0]
    bt = dict(n=ns, offset=offs, params=[psd, psd], dt=[1.0, 1.0], iters=[3, 7], seed=[1, 2], curve_id=[0, 1],
              erdf=Fake(3072), tol=-1.0, prec=agn.AGN_FP32, x_out=Fake(3072), delta_out=Fake(14),
              iters_done=Fake(2, "torch.int32"), ws=Fake(1 << 20, "torch.uint8"))
    lag = dict(n=[100, 50], offset=[0, 100], x=Fake(150), lags=[1, 2, 3], units=agn.AGN_SF_LINEAR, sf2_out=Fake(6),
               rep_out=Fake(3), dm_ref=[0.5, 1.0], lam_cut=0.0, exceed_out=Fake(12, "torch.int64"),
               pairs_out=Fake(6, "torch.int64"), ws=Fake(1 << 20, "torch.uint8"))
    out = []
    for name in ("erdf", "x_out", "delta_out", "iters_done"):
        out.append((agn.agn_lc_generate, one, name))
    for name in ("amp", "x0", "x_out", "delta_out", "iters_done", "rank_out"):
        out.append((agn.agn_lc_iterate, it, name))
    for name in ("erdf", "x_out", "delta_out", "iters_done"):
        out.append((agn.agn_lc_generate_batch, bt, name))
        out.append((agn.agn_batch_plan_create, bt, name))
    for name in ("x", "sf2_out", "rep_out", "exceed_out", "pairs_out"):
        out.append((agn.agn_lag_stats_batch, lag, name))
    pg = dict(n=[1024, 2048], offset=[0, 1024], x=Fake(3072), p_offset=[0, 513], P_out=Fake(513 + 1025))
    for name in ("x", "P_out"):
        out.append((agn.agn_periodogram_batch, pg, name))
    dr = dict(params=agn.pdf_params(agn.AGN_PDF_EQ1), n=1000, seed=1, curve_id=0, out=Fake(1000))
    out.append((agn.agn_pdf_draw, dr, "out"))
    sl = dict(params=agn.pdf_params(agn.AGN_PDF_EQ1), n=1000, n_chains=10, burn=5, seed=1, curve_id=0,
              out=Fake(1000))
    out.append((agn.agn_pdf_slice, sl, "out"))
    ed = dict(params=agn.erdf_params(), n=1000, seed=1, curve_id=0, out=Fake(1000))
    out.append((agn.agn_erdf_draw, ed, "out"))
    sp = dict(params=psd, n=n, dt=1.0, seed=1, curve_id=0, prec=agn.AGN_FP64, amp_out=Fake(n // 2 + 1),
              ws=Fake(1 << 20, "torch.uint8"))
    out.append((agn.agn_psd_spectrum, sp, "amp_out"))
    return out


@pytest.mark.parametrize("fn,kw,name", calls(), ids=lambda v: getattr(v, "__name__", v) if callable(v) else
                         (v if isinstance(v, str) else ""))
def test_short_buffer_is_rejected_before_the_library(fn, kw, name):
    needs_lib()
    kw = dict(kw)
    t = kw[name]
    kw[name] = Fake(t.numel() - 1, t.dtype)
    with pytest.raises(agn.AgnError) as e:
        fn(CTX, **kw)
    assert e.value.code == agn.AGN_EINVAL and str(e.value).startswith(f"agn error -1: {name}:"), str(e.value)


def test_bins_extent_uses_the_bin_count():
    needs_lib()
    nb = agn.agn_log_bin_count(1024, 0.1)
    with pytest.raises(agn.AgnError) as e:
        agn.agn_psd_fit_batch(CTX, [1024, 1024], [1.0, 1.0], [agn.psd_params()] * 2, 0.1, [0, nb],
                              Fake(2 * nb - 1), Fake(8))
    assert "bins:" in str(e.value)
    with pytest.raises(agn.AgnError) as e:
        agn.agn_periodogram_batch(CTX, [1024], [0], Fake(1024), [0], Fake(513), 0.1, [3], Fake(nb + 2))
    assert "bins_out:" in str(e.value)


def undefined_names(path):
    """Names a module loads that it never binds (a coarse static check: any
    binding anywhere in the module counts)."""
    import ast
    import builtins
    tree = ast.parse(open(path).read())
    bound = set(dir(builtins)) | {"__file__", "__name__"}
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            bound.add(node.name)
        elif isinstance(node, ast.Import):
            bound.update(a.asname or a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            bound.update(a.asname or a.name for a in node.names)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, (ast.Store, ast.Del)):
            bound.add(node.id)
        elif isinstance(node, ast.arg):
            bound.add(node.arg)
        elif isinstance(node, ast.ExceptHandler) and node.name:
            bound.add(node.name)
    used = {n.id for n in ast.walk(tree) if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load)}
    return sorted(used - bound)


@pytest.mark.parametrize("rel", ["paper_1909_06374_amd/__init__.py", "paper_1909_06374_amd/serving.py",
                                 "paper_1909_06374_amd/synth.py", "paper_1909_06374_amd/build.py", "bench.py",
                                 "__graft_entry__.py"])
def test_no_undefined_names(rel):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    assert undefined_names(os.path.join(root, rel)) == []


def test_valid_call_reaches_the_stream_lookup():
    """With every buffer valid, the binding gets as far as asking torch for
    the current stream (which fails here without a GPU) and no further."""
    needs_lib()
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(Exception) as e:
        agn.agn_pdf_draw(CTX, agn.pdf_params(agn.AGN_PDF_EQ1), 1000, 1, 0, Fake(1000))
    assert not isinstance(e.value, (NameError, agn.AgnError)), repr(e.value)
