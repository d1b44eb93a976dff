"""Python binding of libbest (include/best.h): the same calls, argument marshalling only.

Every computation happens in the HIP library; this module converts problem dicts, numpy
arrays and torch device tensors into the ABI's structs and pointers.  PyTorch supplies
device memory and the stream.  If the library is not built the first call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi as A
from ._abi import (BEST_AIES, BEST_BF16, BEST_FP16, BEST_FP32, BEST_FP64, BEST_HMC,  # noqa: F401
                   BEST_DE, BEST_MALA, BEST_MH, BEST_NUTS, BEST_NUTS_MAX_DEPTH, PRECISIONS,
                   SAMPLERS)

__all__ = ["BestError", "Ctx", "best_init", "best_logL_grad", "best_step", "best_adapt",
           "best_get_state", "best_set_state", "best_get_whitening", "best_set_whitening",
           "best_set_step_size", "best_set_step_multipliers", "best_reinit",
           "best_get_step_counter",
           "best_set_step_counter",
           "best_set_mlp", "best_logL_param_grad", "best_ess", "best_ess_noalloc", "best_rhat", "best_credible", "best_sliced_wasserstein",
           "best_mlp_nparams", "best_standardise", "best_normalise_inputs",
           "best_importance_weights", "Trainer", "EmulatorFn"]

INITS = {"uniform": A.BEST_INIT_UNIFORM, "replicated": A.BEST_INIT_REPLICATED,
         "gaussian": A.BEST_INIT_GAUSSIAN, "hypersphere": A.BEST_INIT_HYPERSPHERE}


class BestError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _lib():
    return A.load()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch absent
        pass
    return C.c_void_p(None)


def _is_tensor(x):
    try:
        import torch
        return isinstance(x, torch.Tensor)
    except Exception:  # pragma: no cover
        return False


def _tensor_ptr(t, dtype_name):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"expected torch.{dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


class Ctx:
    """Owns a best_ctx handle (best_destroy on close / garbage collection)."""

    def __init__(self, handle, d, n_chains, keep, width=0, n_hidden=0, mlp_coef=0.0,
                 offset=0.0, params=None):
        self.h = handle
        self.d = d
        self.n_chains = n_chains
        self._keep = keep
        # the network's shape and the MLP term's coefficients, as last set on the context
        self.width, self.n_hidden = width, n_hidden
        self.mlp_coef, self.offset = mlp_coef, offset
        self._params = params

    def check(self, rc):
        if rc != A.BEST_OK:
            msg = _lib().best_last_error(self.h)
            raise BestError(rc, (msg or b"").decode() or _lib().best_strerror(rc).decode())

    def close(self):
        if self.h:
            _lib().best_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_struct(prob):
    d = int(prob["d"])
    keep = []

    def arr(v):
        if v is None:
            return None
        a = _f64(v)
        keep.append(a)
        return _dptr(a)

    tw = prob.get("twist")
    ps = A.Problem()
    ps.d = d
    ps.lower, ps.upper = arr(prob["lower"]), arr(prob["upper"])
    ps.gauss_coef = float(prob.get("gauss_coef", 0.0))
    ps.gauss_mean = arr(prob.get("gauss_mean"))
    ps.gauss_prec = arr(prob.get("gauss_prec"))
    ps.twist_u = int(tw["u"]) if tw else -1
    ps.twist_v = int(tw["v"]) if tw else -1
    ps.twist_beta = float(tw["beta"]) if tw else 0.0
    ps.twist_center = float(tw["center"]) if tw else 0.0
    ps.twist_kappa = float(tw["kappa"]) if tw else 0.0
    ps.width, ps.n_hidden = int(prob["width"]), int(prob["n_hidden"])
    ps.mlp_params = arr(prob.get("mlp_params"))
    ps.in_center, ps.in_invscale = arr(prob.get("in_center")), arr(prob.get("in_invscale"))
    ps.mlp_coef, ps.offset = float(prob.get("mlp_coef", 0.0)), float(prob.get("offset", 0.0))
    ps.plain_mode = int(prob.get("plain_mode", 0))
    ps.box_penalty = int(prob.get("box_penalty", 0))
    ps.penalty_width = float(prob.get("penalty_width", 0.01))
    ps.train_lo, ps.train_hi = arr(prob.get("train_lo")), arr(prob.get("train_hi"))
    pl = prob.get("plain")
    if pl is not None and ps.plain_mode != 0:
        pm = A.PlainModel()
        pm.n_bins, pm.n_terms = int(pl["n_bins"]), int(pl["n_terms"])
        pm.xgrid, pm.data, pm.inv_sigma2 = arr(pl["xgrid"]), arr(pl["data"]), arr(pl["inv_sigma2"])
        pm.a, pm.g, pm.p = arr(pl["a"]), arr(pl["g"]), arr(pl["p"])
        pm.k, pm.gamma0 = arr(pl["k"]), arr(pl["gamma0"])
        pm.center, pm.invscale = arr(pl["center"]), arr(pl["invscale"])
        keep.append(pm)
        ps.plain = C.pointer(pm)
    return ps, keep


def best_mlp_nparams(d, width, n_hidden):
    return int(_lib().best_mlp_nparams(d, width, n_hidden))


def best_init(problem, n_chains, precision="fp32", seed=0, init="uniform", init_point=None,
              init_scale=1.0, chains_per_block=0, stream=None) -> Ctx:
    lib = _lib()
    ps, keep = _problem_struct(problem)
    cfg = A.Config()
    cfg.n_chains = int(n_chains)
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.seed = int(seed)
    cfg.init = INITS[init] if isinstance(init, str) else int(init)
    ip = _f64(init_point)
    keep.append(ip)
    cfg.init_point = _dptr(ip)
    cfg.init_scale = float(init_scale)
    cfg.stream = _stream(stream)
    cfg.chains_per_block = int(chains_per_block)
    h = C.c_void_p()
    rc = lib.best_init(C.byref(h), C.byref(ps), C.byref(cfg))
    if rc != A.BEST_OK:
        raise BestError(rc, "best_init failed: " + lib.best_strerror(rc).decode())
    mp = problem.get("mlp_params")
    return Ctx(h, int(problem["d"]), int(n_chains), None, width=int(problem["width"]),
               n_hidden=int(problem["n_hidden"]), mlp_coef=float(problem.get("mlp_coef", 0.0)),
               offset=float(problem.get("offset", 0.0)),
               params=None if mp is None else _f64(mp).copy())


def best_logL_grad(ctx, x, want_grad=True, out=None, aos=False):
    """x: [d][n] float64, or [n][d] with aos=True (numpy -> host path, torch CUDA tensor ->
    device path).  Returns (logL, grad) of the same kind and layout (grad None if not
    wanted)."""
    lib = _lib()
    flags = A.BEST_AOS if aos else 0
    if _is_tensor(x):
        import torch
        n = x.shape[0] if aos else x.shape[1]
        lp = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out[0]
        g = (torch.empty(tuple(x.shape), dtype=torch.float64, device=x.device) if out is None
             else out[1]) if want_grad else None
        ctx.check(lib.best_logL_grad(ctx.h, _tensor_ptr(x, "float64"), n,
                                     _tensor_ptr(lp, "float64"),
                                     _tensor_ptr(g, "float64") if g is not None else None, flags))
        return lp, g
    xa = _f64(x)
    n = xa.shape[0] if aos else xa.shape[1]
    lp = np.empty(n)
    g = np.empty(xa.shape) if want_grad else None
    ctx.check(lib.best_logL_grad(ctx.h, xa.ctypes.data_as(C.c_void_p), n,
                                 lp.ctypes.data_as(C.c_void_p),
                                 g.ctypes.data_as(C.c_void_p) if g is not None else None,
                                 flags | A.BEST_HOST_PTRS))
    return lp, g


def best_step(ctx, sampler, n_steps, eps=0.0, mh_scale=0.0, stretch_a=2.0, n_leapfrog=10,
              thin=1, record=None, adapt_eps=False, target_accept=0.57, max_depth=8,
              de_sigma=0.1):
    """Advance every chain n_steps transitions of sampler "mh", "mala", "hmc", "nuts", "aies"
    or "de".  eps <= 0 uses the context's step size (dual averaging with adapt_eps);
    n_leapfrog: HMC; max_depth: NUTS; stretch_a: AIES; de_sigma: sd of the DE gamma noise.
    record: CUDA float32 tensor [capacity][d][n_chains] or None.  Returns the call's
    statistics as a dict (for NUTS, evals counts the leaves of the trajectories)."""
    lib = _lib()
    p = A.StepParams()
    p.eps, p.mh_scale, p.stretch_a = float(eps), float(mh_scale), float(stretch_a)
    p.n_leapfrog, p.thin = int(n_leapfrog), int(thin)
    if record is not None:
        p.record = C.cast(_tensor_ptr(record, "float32"), C.POINTER(C.c_float))
        p.record_capacity = int(record.shape[0])
    p.adapt_eps = int(bool(adapt_eps))
    p.target_accept = float(target_accept)
    p.max_depth = int(max_depth)
    p.de_sigma = float(de_sigma)
    st = A.StepStats()
    s = SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
    ctx.check(lib.best_step(ctx.h, s, int(n_steps), C.byref(p), C.byref(st)))
    return {k: getattr(st, k) for k, _ in A.StepStats._fields_}


def best_adapt(ctx, samples=None, update_mean=True, reset_da=False, finalize_da=False,
               target_accept=0.0):
    lib = _lib()
    p = A.AdaptParams()
    if samples is not None:
        p.samples = C.cast(_tensor_ptr(samples, "float32"), C.POINTER(C.c_float))
        p.n_samples = int(samples.shape[0])
    p.update_mean, p.reset_da, p.finalize_da = int(update_mean), int(reset_da), int(finalize_da)
    p.target_accept = float(target_accept)
    info = A.AdaptInfo()
    rc = lib.best_adapt(ctx.h, C.byref(p), C.byref(info))
    ctx.check(rc)
    return {k: getattr(info, k) for k, _ in A.AdaptInfo._fields_}


def best_get_state(ctx):
    """Host copies: x [d][n], logL [n], grad [d][n]."""
    x = np.empty((ctx.d, ctx.n_chains))
    lp = np.empty(ctx.n_chains)
    g = np.empty((ctx.d, ctx.n_chains))
    ctx.check(_lib().best_get_state(ctx.h, x.ctypes.data_as(C.c_void_p),
                                    lp.ctypes.data_as(C.c_void_p),
                                    g.ctypes.data_as(C.c_void_p), A.BEST_HOST_PTRS))
    return x, lp, g


def best_set_state(ctx, x, logL=None, grad=None):
    """Host arrays x [d][n] and optionally logL [n] and grad [d][n] (both or neither)."""
    xa = _f64(x)
    assert xa.shape == (ctx.d, ctx.n_chains)
    la, ga = _f64(logL), _f64(grad)
    ctx.check(_lib().best_set_state(ctx.h, xa.ctypes.data_as(C.c_void_p),
                                    la.ctypes.data_as(C.c_void_p) if la is not None else None,
                                    ga.ctypes.data_as(C.c_void_p) if ga is not None else None,
                                    A.BEST_HOST_PTRS))


def best_get_whitening(ctx):
    mu = np.empty(ctx.d)
    L = np.empty((ctx.d, ctx.d))
    ctx.check(_lib().best_get_whitening(ctx.h, _dptr(mu), _dptr(L)))
    return mu, L


def best_set_whitening(ctx, mu, L):
    mu, L = _f64(mu), _f64(L)
    ctx.check(_lib().best_set_whitening(ctx.h, _dptr(mu), _dptr(L)))


def best_set_step_size(ctx, eps):
    ctx.check(_lib().best_set_step_size(ctx.h, float(eps)))


def best_get_step_counter(ctx):
    return int(_lib().best_get_step_counter(ctx.h))


def best_set_step_counter(ctx, step):
    ctx.check(_lib().best_set_step_counter(ctx.h, int(step)))


def best_reinit(ctx, init="gaussian", point=None, scale=1.0):
    """Re-initialise every walker (uniform / replicated / gaussian or hypersphere around
    point with the current whitening factor)."""
    pa = _f64(point)
    ctx.check(_lib().best_reinit(ctx.h, INITS[init] if isinstance(init, str) else int(init),
                                 _dptr(pa), float(scale)))


def best_set_step_multipliers(ctx, m):
    """Per-dimension step multipliers (host [d]) for MALA and MH; None removes them."""
    ma = _f64(m)
    ctx.check(_lib().best_set_step_multipliers(ctx.h, _dptr(ma)))


def best_set_mlp(ctx, params, mlp_coef, offset=0.0):
    p = _f64(params)
    ctx.check(_lib().best_set_mlp(ctx.h, _dptr(p), float(mlp_coef), float(offset)))
    ctx._params, ctx.mlp_coef, ctx.offset = p.copy(), float(mlp_coef), float(offset)


def best_logL_param_grad(ctx, x, upstream=None, out=None):
    """Gradient of sum_c upstream[c] * log pi(x[:, c]) with respect to the flat MLP
    parameters.  x: CUDA float64 [d][n]; upstream: CUDA float64 [n] or None (ones).
    Returns a CUDA float64 tensor [nparams]."""
    import torch
    d, n = x.shape
    npar = best_mlp_nparams(d, ctx.width, ctx.n_hidden)
    g = torch.empty(npar, dtype=torch.float64, device=x.device) if out is None else out
    ctx.check(_lib().best_logL_param_grad(
        ctx.h, _tensor_ptr(x, "float64"), int(n),
        _tensor_ptr(upstream, "float64") if upstream is not None else None,
        _tensor_ptr(g, "float64")))
    return g


ESS_FLAGS = {A.BEST_ESS_OK: "ok", A.BEST_ESS_UNTRUNCATED: "untruncated",
             A.BEST_ESS_FROZEN: "frozen"}


def best_ess(ctx, record, n=None, flags=False):
    """record: CUDA float32 tensor [T][d][n_chains]; returns per-parameter ESS (numpy), and
    with flags=True also the per-parameter BEST_ESS_* flags (int32 numpy)."""
    T = int(record.shape[0]) if n is None else int(n)
    out = np.empty(ctx.d)
    fl = np.zeros(ctx.d, dtype=np.int32)
    ctx.check(_lib().best_ess(ctx.h, _tensor_ptr(record, "float32"), T, _dptr(out),
                              fl.ctypes.data_as(C.c_void_p)))
    return (out, fl) if flags else out


def best_ess_noalloc(ctx, record, n=None, flags=False):
    """best_ess through the entry point that allocates no device memory (fixed per-GPU
    scratch; d * ceil(n_chains / 64) * 64 <= 2^20)."""
    T = int(record.shape[0]) if n is None else int(n)
    out = np.empty(ctx.d)
    fl = np.zeros(ctx.d, dtype=np.int32)
    ctx.check(_lib().best_ess_noalloc(ctx.h, _tensor_ptr(record, "float32"), T, _dptr(out),
                                      fl.ctypes.data_as(C.c_void_p)))
    return (out, fl) if flags else out


def _record(rec):
    if rec.dim() != 3:
        raise ValueError("expected a record [T][d][n_chains]")
    return _tensor_ptr(rec, "float32"), int(rec.shape[0]), int(rec.shape[2])


def _whitening(whitening):
    if whitening is None:
        return None, None
    mu, L = whitening
    return _f64(mu), _f64(L)


def best_rhat(ctx, record):
    """Multivariate R - 1 (Sec. 4.1) of a CUDA float32 record [T][d][n_chains]."""
    p, T, n = _record(record)
    out = np.empty(1)
    ctx.check(_lib().best_rhat(ctx.h, p, T, n, _dptr(out)))
    return float(out[0])


def best_credible(ctx, record, alpha, whitening=None, ref=None):
    """Equal-tailed credible limits at level alpha of every parameter, and with
    ref = (lo0, hi0) the credible metric of Sec. 4.1.  whitening = (mu, L) or None.
    Returns (lo, hi, metric or None)."""
    p, T, n = _record(record)
    mu, L = _whitening(whitening)
    lo, hi = np.empty(ctx.d), np.empty(ctx.d)
    r_lo, r_hi = (None, None) if ref is None else (_f64(ref[0]), _f64(ref[1]))
    m = np.empty(1) if ref is not None else None
    ctx.check(_lib().best_credible(ctx.h, p, T, n, float(alpha), _dptr(mu), _dptr(L),
                                   _dptr(r_lo), _dptr(r_hi), _dptr(lo), _dptr(hi), _dptr(m)))
    return lo, hi, (float(m[0]) if m is not None else None)


def best_sliced_wasserstein(ctx, rec_a, rec_b, n_proj=500, proj_seed=0x5EED, whitening=None):
    """Sliced Wasserstein distance (Sec. 4.1) between two CUDA float32 records."""
    pa, Ta, na = _record(rec_a)
    pb, Tb, nb = _record(rec_b)
    mu, L = _whitening(whitening)
    out = np.empty(1)
    ctx.check(_lib().best_sliced_wasserstein(ctx.h, pa, Ta, na, pb, Tb, nb, int(n_proj),
                                             int(proj_seed), _dptr(mu), _dptr(L), _dptr(out)))
    return float(out[0])


def best_standardise(y, stream=None):
    """y: CUDA float64 tensor [n] -> (float32 tensor of standardised values, mean, std)."""
    import torch
    out = torch.empty(y.shape[0], dtype=torch.float32, device=y.device)
    ms = np.empty(2)
    rc = _lib().best_standardise(_tensor_ptr(y, "float64"), int(y.shape[0]),
                                 _tensor_ptr(out, "float32"), _dptr(ms), _stream(stream))
    if rc != A.BEST_OK:
        raise BestError(rc, "best_standardise failed")
    return out, float(ms[0]), float(ms[1])


def best_normalise_inputs(x, center, invscale, stream=None):
    """x: CUDA float64 [d][n] -> CUDA float32 [n][d] of (x - center) * invscale."""
    import torch
    d, n = x.shape
    t = torch.empty((n, d), dtype=torch.float32, device=x.device)
    c, s = _f64(center), _f64(invscale)
    rc = _lib().best_normalise_inputs(_tensor_ptr(x, "float64"), int(n), int(d), _dptr(c),
                                      _dptr(s), _tensor_ptr(t, "float32"), _stream(stream))
    if rc != A.BEST_OK:
        raise BestError(rc, "best_normalise_inputs: " + _lib().best_strerror(rc).decode())
    return t


def best_importance_weights(logl_plain, logl_emu, stream=None):
    """CUDA float64 tensors [n] -> (normalised weights tensor, Kish ESS)."""
    import torch
    w = torch.empty_like(logl_plain)
    kish = np.empty(1)
    rc = _lib().best_importance_weights(_tensor_ptr(logl_plain, "float64"),
                                        _tensor_ptr(logl_emu, "float64"), int(w.shape[0]),
                                        _tensor_ptr(w, "float64"), _dptr(kish), _stream(stream))
    if rc != A.BEST_OK:
        raise BestError(rc, "best_importance_weights failed")
    return w, float(kish[0])


class Trainer:
    """best_trainer_* calls: FP64 master weights + Adam on the device."""

    def __init__(self, d, width, n_hidden, init_params, precision="fp32", stream=None):
        self.lib = _lib()
        self.p0 = _f64(init_params)
        self.np = best_mlp_nparams(d, width, n_hidden)
        assert self.p0.size == self.np
        self.h = C.c_void_p()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        rc = self.lib.best_trainer_create(C.byref(self.h), d, width, n_hidden, _dptr(self.p0),
                                          prec, _stream(stream))
        if rc != A.BEST_OK:
            raise BestError(rc, "best_trainer_create failed")

    def check(self, rc):
        if rc != A.BEST_OK:
            raise BestError(rc, (self.lib.best_trainer_last_error(self.h) or b"").decode())

    def epoch(self, t_in, y, perm, batch, lr0, lr1, step0, total_steps):
        loss = C.c_double()
        self.check(self.lib.best_train_epoch(
            self.h, _tensor_ptr(t_in, "float32"), _tensor_ptr(y, "float32"), int(t_in.shape[0]),
            _tensor_ptr(perm, "int32"), int(batch), float(lr0), float(lr1), int(step0),
            int(total_steps), C.byref(loss)))
        return loss.value

    def grad(self, t_in, y):
        g = np.empty(self.np)
        loss = C.c_double()
        self.check(self.lib.best_train_grad(self.h, _tensor_ptr(t_in, "float32"),
                                            _tensor_ptr(y, "float32"), int(t_in.shape[0]),
                                            _dptr(g), C.byref(loss)))
        return loss.value, g

    def params(self):
        out = np.empty(self.np)
        self.check(self.lib.best_trainer_get_params(self.h, _dptr(out)))
        return out

    def close(self):
        if self.h:
            self.lib.best_trainer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _emulator_fn():
    import torch

    def sync_params(ctx, p):
        """Load the MLP parameters p (float64 numpy) into the context if they differ."""
        if ctx._params is None or ctx._params.shape != p.shape or not np.array_equal(ctx._params, p):
            best_set_mlp(ctx, p, ctx.mlp_coef, ctx.offset)

    class EmulatorFn(torch.autograd.Function):
        """log pi(x) of a context's target, differentiable with respect to the points and,
        when given, the flat MLP parameters.  Backward runs the library's hand-written
        kernels: the input gradient of best_logL_grad and the weight gradients of
        best_logL_param_grad.  x: CUDA float64 [d][n]; params: float64 [nparams] (any
        device) or None (the context's current network); returns [n]."""

        @staticmethod
        def forward(fctx, ctx, x, params=None):
            p = None
            if params is not None:
                p = params.detach().to("cpu", torch.float64).numpy().copy()
                sync_params(ctx, p)
            xd = x.detach().contiguous()
            lp, g = best_logL_grad(ctx, xd, want_grad=True)
            fctx.ctx, fctx.p, fctx.params_like = ctx, p, params
            fctx.save_for_backward(g, xd)
            return lp

        @staticmethod
        def backward(fctx, grad_out):
            g, xd = fctx.saved_tensors
            go = grad_out.detach().to(torch.float64).contiguous()
            gx = g * go[None, :] if fctx.needs_input_grad[1] else None
            gp = None
            if fctx.p is not None and fctx.needs_input_grad[2]:
                sync_params(fctx.ctx, fctx.p)  # the network of this forward
                gp = best_logL_param_grad(fctx.ctx, xd, go).to(fctx.params_like.device)
            return None, gx, gp

    return EmulatorFn


class _Lazy:
    def __getattr__(self, item):
        return getattr(_emulator_fn(), item)


EmulatorFn = _Lazy()
