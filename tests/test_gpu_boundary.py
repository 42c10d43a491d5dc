"""Boundary entry points beyond the time step, through the C ABI: contexts
made from device arrays (lbe_init_device), fields written to device memory
(lbe_fields_device), the Poisson stopping rule changed on a live context
(lbe_set_solver), and a step whose solve fails going back to its start."""
import ctypes as C

import numpy as np
import pytest

import gpu_cases as G
import oracle
import paper_1907_04732_amd as lbe

pytestmark = pytest.mark.gpu

FORMS = {
    "fp64-sor": dict(precision=lbe.FP64, poisson=lbe.SOR4),
    "fp32-mg": dict(precision=lbe.FP32_MIXED, poisson=lbe.MG, flags=lbe.EXTRAPOLATE),
}


def _inputs(name="random_6x10x14_k3"):
    kw, shape, t, ps, n0, nref, _, _ = G.case(name)
    rng = np.random.default_rng(17)
    f0 = G._rest(t) * (1 + 1e-3 * rng.standard_normal((19, t.size)))
    return kw, shape, t, ps, np.asarray(n0).reshape(len(kw["z"]), -1), np.asarray(nref, float), f0


def _params(kw, shape, form, **extra):
    k = dict(kw)
    k["flags"] = k.get("flags", 0) | FORMS[form].get("flags", 0)
    f = {a: b for a, b in FORMS[form].items() if a != "flags"}
    return lbe.make_params(shape, **k, tol=1e-11, max_iter=100000, **f, **extra)


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("form", list(FORMS))
def test_init_from_device_arrays_matches_host_init(form):
    import torch

    kw, shape, t, ps, n0, nref, f0 = _inputs()
    dev = torch.device("cuda", 0)
    h = lbe.Lbe(_params(kw, shape, form), t, ps, n0, nref, f0)
    d = lbe.Lbe(_params(kw, shape, form), torch.as_tensor(t, device=dev),
                torch.as_tensor(ps, device=dev), torch.as_tensor(n0, device=dev),
                torch.as_tensor(nref, device=dev), torch.as_tensor(f0, device=dev))
    assert d.ne == h.ne
    _same(h.fields(), d.fields())
    h.step(12)
    d.step(12)
    _same(h.fields(), d.fields())
    assert np.array_equal(h.qhist(), d.qhist())
    # n_ref alone: uniform concentrations, rest populations
    h2 = lbe.Lbe(_params(kw, shape, form), t, ps, None, nref)
    d2 = lbe.Lbe(_params(kw, shape, form), torch.as_tensor(t, device=dev),
                 torch.as_tensor(ps, device=dev), None, torch.as_tensor(nref, device=dev))
    h2.step(3)
    d2.step(3)
    _same(h2.fields(), d2.fields())


@pytest.mark.parametrize("form", list(FORMS))
def test_fields_to_device_memory_match_host_copies(form):
    import torch

    kw, shape, t, ps, n0, nref, f0 = _inputs()
    g = lbe.Lbe(_params(kw, shape, form), t, ps, n0, nref, f0)
    g.step(7)
    host = g.fields()
    dev = g.fields(device=torch.device("cuda", 0))
    for k in host:
        assert np.array_equal(host[k], dev[k].cpu().numpy()), k
    part = g.fields(f=False, device=torch.device("cuda", 0))
    assert "f" not in part and np.array_equal(part["n"].cpu().numpy(), host["n"])


def test_host_pointers_are_rejected_where_device_memory_is_expected():
    kw, shape, t, ps, n0, nref, f0 = _inputs()
    lib = lbe.load()
    p = _params(kw, shape, "fp64-sor")
    h = C.c_void_p()
    tt = np.ascontiguousarray(t, np.uint8)
    rc = lib.lbe_init_device(C.byref(p), C.c_void_p(tt.ctypes.data), C.c_void_p(ps.ctypes.data),
                             None, C.c_void_p(nref.ctypes.data), None, C.byref(h))
    assert rc == lbe.EINVAL and not h.value
    g = lbe.Lbe(p, t, ps, n0, nref)
    buf = np.empty(g.N)
    rc = lib.lbe_fields_device(g.h, C.c_void_p(buf.ctypes.data), None, None, None)
    assert rc == lbe.EINVAL
    assert b"device memory" in lib.lbe_last_error(g.h)


def test_set_solver_fixed_count_and_errors():
    kw, shape, t, ps, n0, nref, f0 = _inputs()
    g = lbe.Lbe(_params(kw, shape, "fp64-sor"), t, ps, n0, nref)
    g.set_solver(tol=0.0, max_iter=7)
    g.step(2)
    assert g.totals()["poisson_iters"] == 7
    for bad in (dict(tol=float("nan")), dict(tol=float("inf")), dict(max_iter=-1)):
        with pytest.raises(lbe.LbeError) as e:
            g.set_solver(**bad)
        assert e.value.code == lbe.EINVAL
    g.step(1)
    assert g.totals()["poisson_iters"] == 7


def _snapshot(g):
    return g.fields(), g.qhist(), g.totals()["step"]


def _fail_one_step(g):
    tol, max_iter = g.p.tol, g.p.max_iter
    before = _snapshot(g)
    g.set_solver(tol=1e-15, max_iter=1)
    with pytest.raises(lbe.LbeError) as e:
        g.step(3)
    assert e.value.code == lbe.ENOCONV
    tot = g.totals()
    assert tot["poisson_iters"] == 1 and tot["poisson_resid"] > 1e-15
    after = _snapshot(g)
    _same(before[0], after[0])
    assert np.array_equal(before[1], after[1]) and before[2] == after[2]
    g.set_solver(tol=tol, max_iter=max_iter)


def test_failed_step_goes_back_to_its_start_fp64():
    """FP64 SOR: the rewind restores the state bit for bit, and after the
    limit is raised the retried steps follow the uninterrupted trajectory
    exactly (the residual checks run on a fixed schedule) and match the
    oracle put through the same failure."""
    kw, shape, t, ps, n0, nref, f0 = _inputs("slab_2x2x18_k1")
    p = _params(kw, shape, "fp64-sor")
    g = lbe.Lbe(p, t, ps, n0, nref, f0)
    ref = lbe.Lbe(_params(kw, shape, "fp64-sor"), t, ps, n0, nref, f0)
    o = oracle.Oracle(oracle.make_params(shape, **kw, tol=p.tol, max_iter=p.max_iter,
                                         check_every=p.check_every), t, ps, n0, nref, f0)
    g.step(4)
    o.step(4)
    _fail_one_step(g)
    o.set_solver(1e-15, 1)
    with pytest.raises(oracle.OracleError):
        o.step(3)
    o.set_solver(p.tol, p.max_iter)
    g.step(3)
    o.step(3)
    ref.step(7)
    _same(g.fields(), ref.fields())
    assert np.array_equal(g.qhist(), ref.qhist())
    fo, fg = o.fields(), g.fields()
    for k in ("phi", "n", "f"):
        assert np.abs(fg[k] - fo[k]).max() <= 1e-11 * np.abs(fo[k]).max(), k
    assert np.abs(g.qhist() - o.qhist()).max() <= 1e-11 * np.abs(o.qhist()).max()


def test_failed_step_goes_back_to_its_start_mixed_multigrid():
    """Mixed form, multigrid with the extrapolated start: the rewind restores
    the state bit for bit; the retried step starts from a linear rather than
    quadratic extrapolation, so it converges to the same tolerance but not
    to the same bits."""
    kw, shape, t, ps, n0, nref, f0 = _inputs()
    g = lbe.Lbe(_params(kw, shape, "fp32-mg"), t, ps, n0, nref, f0)
    ref = lbe.Lbe(_params(kw, shape, "fp32-mg"), t, ps, n0, nref, f0)
    g.step(5)
    _fail_one_step(g)
    g.step(3)
    ref.step(8)
    a, b = g.fields(), ref.fields()
    dv = np.ptp(ps[t > 0])
    assert g.totals()["poisson_resid"] <= 1e-11
    assert np.abs(a["phi"] - b["phi"]).max() <= 1e-8 * dv
    nscale = np.abs(b["n"] - b["n"].mean(1, keepdims=True)).max()
    assert np.abs(a["n"] - b["n"]).max() <= 1e-6 * nscale
    assert g.qhist().shape == ref.qhist().shape


@pytest.mark.parametrize("form", list(FORMS))
def test_pass_block_size_does_not_change_results(form, monkeypatch):
    """The step passes compute every site on its own, so the block size the
    context picks for them (timed at creation, or fixed by LBE_PASS_BLOCK)
    changes no bit of the trajectory."""
    kw, shape, t, ps, n0, nref, f0 = _inputs()
    out = []
    for tb in ("128", "256", "512"):
        monkeypatch.setenv("LBE_PASS_BLOCK", tb)
        g = lbe.Lbe(_params(kw, shape, form), t, ps, n0, nref, f0)
        g.step(9)
        out.append((g.fields(), g.qhist()))
        g.close()
    for fa, qa in out[1:]:
        _same(out[0][0], fa)
        assert np.array_equal(out[0][1], qa)
