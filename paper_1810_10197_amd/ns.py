"""Thin ctypes binding of the C ABI in include/ns.h (argument marshalling only).

The module-level functions carry the C names (ns_init, ns_rhs, ...) and
take plain integers for device pointers; :class:`Solver` wraps them with
PyTorch tensors, which provide the device memory (state, right-hand side,
workspace) and the stream.  Every numerical step runs in the HIP library;
if ``libns.so`` is missing this module raises on import.
"""
import ctypes
import os

import numpy as np
# torch first: libns.so then binds to the HIP runtime torch already loaded
# (same soname), so streams and device pointers from torch are valid in it.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libns.so")

NS_OK = 0
NS_STEP_REJECTED = 1
NS_ERR_ARG = -1
NS_ERR_HIP = -2
NS_ERR_NOMEM = -3
NS_ERR_NONFINITE = -4
NS_ERR_STEPFAIL = -5
NS_ERR_UNSUPPORTED = -6
NS_ERR_STATE = -7
NS_ERR_SCRATCH = -8
NS_FP32 = 0
NS_FP64 = 1
NS_CTRL_PI = 0
NS_CTRL_MLP = 1
NS_FORCE_COMMIT = 1
NS_INTEGRATE_HOST = 0x100
NS_METHOD_DP5 = 0x200
NS_INTEGRATE_RESUME = 0x400
NS_MLP_NPARAM = 5569
NS_MLP_NWEIGHTS = 5609
NS_STATIC_SCRATCH_BYTES = 64 << 20
NS_STATIC_MAX_BATCH = 64

EXPORTS = ["ns_workspace_bytes", "ns_init", "ns_set_state", "ns_get_state", "ns_set_nu",
           "ns_rhs", "ns_step_rk4", "ns_step_bs5", "ns_step_dp5", "ns_integrate", "ns_get_time",
           "ns_set_time", "ns_diagnostics", "ns_refresh_rhs", "ns_mlp_set_weights",
           "ns_mlp_get_weights", "ns_mlp_forward", "ns_mlp_grad", "ns_mlp_train_batch",
           "ns_mlp_reset_optimizer", "ns_mlp_collect", "ns_mlp_rows", "ns_mlp_push_rows",
           "ns_mlp_fit_stats", "ns_checkpoint_bytes", "ns_checkpoint_save", "ns_checkpoint_load",
           "ns_save", "ns_load",
           "ns_mlp_train", "ns_autotune", "ns_tune_get", "ns_tune_set", "ns_profile_start",
           "ns_profile_stop", "ns_strerror", "ns_free", "ns_rhs_static", "ns_rhs_static_bytes", "ns_profile_mode"]
NS_NTUNE = 6
NS_TUNE_MAXV = 13
NS_DEALIAS = {"2/3": 0, "3/2": 1}
PROF_NAMES = ["zinv", "yinv", "xpass", "yfwd", "zfwd", "combine", "reduce", "other", "slab", "rhs"]


class NsConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("batch", ctypes.c_int),
                ("rhs_precision", ctypes.c_int), ("scalar", ctypes.c_int),
                ("ri", ctypes.c_double), ("kappa", ctypes.c_double),
                ("force_kf", ctypes.c_double), ("force_e0", ctypes.c_double),
                ("dealias", ctypes.c_int)]


class NsStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h_next", ctypes.c_double),
                ("last_err", ctypes.c_double), ("n_rhs", ctypes.c_longlong),
                ("n_accept", ctypes.c_longlong), ("n_reject", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


NS_NPROF = 10


class NsKernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NS_NPROF), ("count", ctypes.c_longlong * NS_NPROF)]


if not os.path.exists(LIB_PATH):
    raise ImportError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)
_FP = ctypes.POINTER(ctypes.c_float)
_sig = {
    "ns_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(NsConfig)]),
    "ns_init": (_I, [ctypes.POINTER(NsConfig), _DP, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "ns_set_state": (_I, [_P, _P]),
    "ns_get_state": (_I, [_P, _P]),
    "ns_set_nu": (_I, [_P, _DP]),
    "ns_rhs": (_I, [_P, _P, _P]),
    "ns_step_rk4": (_I, [_P, _D]),
    "ns_step_bs5": (_I, [_P, _D, _D, _D, _I, _DP]),
    "ns_step_dp5": (_I, [_P, _D, _D, _D, _I, _DP]),
    "ns_integrate": (_I, [_P, _D, _D, _D, _D, _I, ctypes.POINTER(NsStats)]),
    "ns_get_time": (_I, [_P, _DP]),
    "ns_set_time": (_I, [_P, _DP]),
    "ns_diagnostics": (_I, [_P, _DP, _DP, _DP]),
    "ns_refresh_rhs": (_I, [_P]),
    "ns_mlp_set_weights": (_I, [_P, _FP]),
    "ns_mlp_get_weights": (_I, [_P, _FP]),
    "ns_mlp_forward": (_I, [_P, _P, _I, _P]),
    "ns_mlp_grad": (_I, [_P, _P, _P, _I, _FP, _FP]),
    "ns_mlp_train_batch": (_I, [_P, _P, _P, _I, ctypes.c_float, _FP]),
    "ns_mlp_reset_optimizer": (_I, [_P]),
    "ns_mlp_collect": (_I, [_P, _I]),
    "ns_mlp_rows": (_I, [_P, _FP, _FP, _I, ctypes.POINTER(ctypes.c_longlong)]),
    "ns_mlp_push_rows": (_I, [_P, _FP, _FP, _I]),
    "ns_mlp_fit_stats": (_I, [_P]),
    "ns_mlp_train": (_I, [_P, _I, _I, ctypes.c_float, ctypes.c_ulonglong, _FP]),
    "ns_autotune": (_I, [_P, _I, _DP]),
    "ns_tune_get": (_I, [_P, ctypes.POINTER(ctypes.c_int)]),
    "ns_tune_set": (_I, [_P, ctypes.POINTER(ctypes.c_int)]),
    "ns_profile_start": (_I, [_P]),
    "ns_profile_stop": (_I, [_P, ctypes.POINTER(NsKernelTimes)]),
    "ns_strerror": (ctypes.c_char_p, [_I]),
    "ns_checkpoint_bytes": (ctypes.c_size_t, [_P]),
    "ns_checkpoint_save": (_I, [_P, _P, ctypes.c_size_t]),
    "ns_checkpoint_load": (_I, [_P, _P, ctypes.c_size_t]),
    "ns_save": (_I, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "ns_load": (_I, [_P, _P, ctypes.c_size_t]),
    "ns_free": (None, [_P]),
    "ns_rhs_static": (_I, [ctypes.POINTER(NsConfig), _DP, _P, _P, _P]),
    "ns_rhs_static_bytes": (ctypes.c_size_t, [ctypes.POINTER(NsConfig)]),
    "ns_profile_mode": (_I, [_P, _I]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class NsError(RuntimeError):
    def __init__(self, status, where):
        super().__init__("%s: %s (%d)" % (where, ns_strerror(status), status))
        self.status = status


def _dptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def _fptr(a):
    return a.ctypes.data_as(_FP) if a is not None else None


def _check(status, where, ok=(NS_OK,)):
    if status not in ok:
        raise NsError(status, where)
    return status


# ---------------------------------------------------------------- C names
def ns_strerror(status):
    return _lib.ns_strerror(int(status)).decode()


def ns_workspace_bytes(cfg):
    return int(_lib.ns_workspace_bytes(ctypes.byref(cfg)))


def ns_init(cfg, nu, workspace_ptr, workspace_bytes, stream_ptr):
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    h = _P()
    _check(_lib.ns_init(ctypes.byref(cfg), _dptr(nu), _P(workspace_ptr), workspace_bytes,
                        _P(stream_ptr), ctypes.byref(h)), "ns_init")
    return h


def ns_set_state(h, uhat_ptr):
    return _check(_lib.ns_set_state(h, _P(uhat_ptr)), "ns_set_state")


def ns_get_state(h, uhat_ptr):
    return _check(_lib.ns_get_state(h, _P(uhat_ptr)), "ns_get_state")


def ns_set_nu(h, nu):
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    return _check(_lib.ns_set_nu(h, _dptr(nu)), "ns_set_nu")


def ns_rhs(h, uhat_ptr, f_ptr):
    return _check(_lib.ns_rhs(h, _P(uhat_ptr), _P(f_ptr)), "ns_rhs")


def ns_step_rk4(h, dt):
    return _check(_lib.ns_step_rk4(h, float(dt)), "ns_step_rk4")


def ns_step_bs5(h, dt, atol, rtol, flags, err_out):
    return _check(_lib.ns_step_bs5(h, float(dt), float(atol), float(rtol), int(flags),
                                   _dptr(err_out)), "ns_step_bs5",
                  ok=(NS_OK, NS_STEP_REJECTED))


def ns_step_dp5(h, dt, atol, rtol, flags, err_out):
    return _check(_lib.ns_step_dp5(h, float(dt), float(atol), float(rtol), int(flags),
                                   _dptr(err_out)), "ns_step_dp5",
                  ok=(NS_OK, NS_STEP_REJECTED))


def ns_integrate(h, t_end, h0, atol, rtol, controller, stats_out):
    return _check(_lib.ns_integrate(h, float(t_end), float(h0), float(atol), float(rtol),
                                    int(controller), stats_out), "ns_integrate")


def ns_get_time(h, t_out):
    return _check(_lib.ns_get_time(h, _dptr(t_out)), "ns_get_time")


def ns_set_time(h, t):
    t = np.ascontiguousarray(t, dtype=np.float64)
    return _check(_lib.ns_set_time(h, _dptr(t)), "ns_set_time")


def ns_diagnostics(h, e_out, eps_out, shells_out):
    return _check(_lib.ns_diagnostics(h, _dptr(e_out), _dptr(eps_out), _dptr(shells_out)),
                  "ns_diagnostics")


def ns_refresh_rhs(h):
    return _check(_lib.ns_refresh_rhs(h), "ns_refresh_rhs")


def ns_mlp_set_weights(h, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    if w.size != NS_MLP_NWEIGHTS:
        raise ValueError("expected %d weights" % NS_MLP_NWEIGHTS)
    return _check(_lib.ns_mlp_set_weights(h, _fptr(w)), "ns_mlp_set_weights")


def ns_mlp_get_weights(h, out):
    return _check(_lib.ns_mlp_get_weights(h, _fptr(out)), "ns_mlp_get_weights")


def ns_mlp_forward(h, x_ptr, n, y_ptr):
    return _check(_lib.ns_mlp_forward(h, _P(x_ptr), int(n), _P(y_ptr)), "ns_mlp_forward")


def ns_mlp_grad(h, x_ptr, t_ptr, n, grad_out, loss_out):
    return _check(_lib.ns_mlp_grad(h, _P(x_ptr), _P(t_ptr), int(n), _fptr(grad_out),
                                   _fptr(loss_out)), "ns_mlp_grad")


def ns_mlp_train_batch(h, x_ptr, t_ptr, n, lr, loss_out):
    return _check(_lib.ns_mlp_train_batch(h, _P(x_ptr), _P(t_ptr), int(n), float(lr),
                                          _fptr(loss_out)), "ns_mlp_train_batch")


def ns_mlp_reset_optimizer(h):
    return _check(_lib.ns_mlp_reset_optimizer(h), "ns_mlp_reset_optimizer")


def ns_mlp_collect(h, enable):
    return _check(_lib.ns_mlp_collect(h, int(bool(enable))), "ns_mlp_collect")


def ns_mlp_rows(h, x_out, y_out, max_rows):
    cnt = ctypes.c_longlong(0)
    _check(_lib.ns_mlp_rows(h, _fptr(x_out), _fptr(y_out), int(max_rows), ctypes.byref(cnt)),
           "ns_mlp_rows")
    return cnt.value


def ns_mlp_push_rows(h, x, y):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return _check(_lib.ns_mlp_push_rows(h, _fptr(x), _fptr(y), int(y.size)), "ns_mlp_push_rows")


def ns_mlp_fit_stats(h):
    return _check(_lib.ns_mlp_fit_stats(h), "ns_mlp_fit_stats")


def ns_mlp_train(h, iters, batch, lr, seed, loss_out):
    return _check(_lib.ns_mlp_train(h, int(iters), int(batch), float(lr), int(seed),
                                    _fptr(loss_out)), "ns_mlp_train")


def ns_autotune(h, reps, ms_out):
    return _check(_lib.ns_autotune(h, int(reps), _dptr(ms_out)), "ns_autotune")


def ns_tune_get(h):
    v = (ctypes.c_int * NS_NTUNE)()
    _check(_lib.ns_tune_get(h, v), "ns_tune_get")
    return list(v)


def ns_tune_set(h, variants):
    v = (ctypes.c_int * NS_NTUNE)(*[int(x) for x in variants])
    return _check(_lib.ns_tune_set(h, v), "ns_tune_set")


def ns_profile_start(h):
    return _check(_lib.ns_profile_start(h), "ns_profile_start")


def ns_profile_mode(h, mode):
    return _check(_lib.ns_profile_mode(h, int(mode)), "ns_profile_mode")


def ns_profile_stop(h, out):
    return _check(_lib.ns_profile_stop(h, ctypes.byref(out)), "ns_profile_stop")


def ns_free(h):
    _lib.ns_free(h)


def ns_rhs_static(cfg, nu, uhat_ptr, f_ptr, stream_ptr):
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    return _check(_lib.ns_rhs_static(ctypes.byref(cfg), _dptr(nu), _P(uhat_ptr), _P(f_ptr),
                                     _P(stream_ptr)), "ns_rhs_static")


def ns_rhs_static_bytes(cfg):
    return int(_lib.ns_rhs_static_bytes(ctypes.byref(cfg)))


# ---------------------------------------------------------------- wrapper
class Solver:
    """One solver instance on a CUDA/HIP device, memory owned by torch."""

    def __init__(self, dim=3, n=32, batch=1, nu=0.0, rhs_precision="fp32", scalar=0,
                 ri=0.0, kappa=0.0, force_kf=0.0, force_e0=0.0, device="cuda", dealias="2/3"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        prec = {"fp32": NS_FP32, "fp64": NS_FP64}[rhs_precision]
        self.cfg = NsConfig(dim, n, batch, prec, scalar, ri, kappa, force_kf, force_e0,
                            NS_DEALIAS[dealias])
        nbytes = ns_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise ValueError("unsupported configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (batch,)).copy()
        self.handle = ns_init(self.cfg, nu, self._ws_ptr, nbytes, self.stream.cuda_stream)
        self.batch = batch
        self.dim = dim
        self.n = n
        self.ncomp = 3 if dim == 3 else (3 if scalar else 2)
        self.shape = ((batch, self.ncomp) + (n,) * (dim - 1) + (n // 2 + 1,))

    def _tensor(self, x):
        t = self.torch
        if isinstance(x, np.ndarray):
            x = t.from_numpy(np.ascontiguousarray(x, dtype=np.complex128))
        x = x.to(device=self.device, dtype=t.complex128).contiguous()
        if tuple(x.shape) != self.shape:
            # one member may come without its batch axis; nothing else is reshaped
            if self.batch == 1 and tuple(x.shape) == self.shape[1:]:
                x = x.reshape(self.shape)
            else:
                raise ValueError("state shape %s, expected %s" % (tuple(x.shape), self.shape))
        return x

    def set_state(self, uhat):
        x = self._tensor(uhat)
        ns_set_state(self.handle, x.data_ptr())
        self.stream.synchronize()

    def get_state(self):
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        ns_get_state(self.handle, out.data_ptr())
        self.stream.synchronize()
        return out

    def rhs(self, uhat):
        x = self._tensor(uhat)
        out = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        ns_rhs(self.handle, x.data_ptr(), out.data_ptr())
        self.stream.synchronize()
        return out

    def set_nu(self, nu):
        ns_set_nu(self.handle, np.broadcast_to(np.asarray(nu, dtype=np.float64), (self.batch,)))

    def step_rk4(self, h):
        ns_step_rk4(self.handle, h)

    def step_bs5(self, h, atol, rtol, force=False):
        errs = np.zeros(self.batch)
        st = ns_step_bs5(self.handle, h, atol, rtol, NS_FORCE_COMMIT if force else 0, errs)
        return st, errs

    def step_dp5(self, h, atol, rtol, force=False):
        errs = np.zeros(self.batch)
        st = ns_step_dp5(self.handle, h, atol, rtol, NS_FORCE_COMMIT if force else 0, errs)
        return st, errs

    def integrate(self, t_end, h0, atol, rtol, controller="pi", graph=True, method="bs5",
                  resume=False):
        stats = (NsStats * self.batch)()
        ctl = {"pi": NS_CTRL_PI, "mlp": NS_CTRL_MLP}[controller]
        if not graph:
            ctl |= NS_INTEGRATE_HOST
        if resume:
            ctl |= NS_INTEGRATE_RESUME
        if method == "dp5":
            ctl |= NS_METHOD_DP5
        elif method != "bs5":
            raise ValueError("method must be 'bs5' or 'dp5'")
        ns_integrate(self.handle, t_end, h0, atol, rtol, ctl, stats)
        return [s.as_dict() for s in stats]

    # ---- checkpoint / resume
    def checkpoint(self):
        """The solver's checkpoint as a numpy uint8 array (host memory)."""
        nbytes = _lib.ns_checkpoint_bytes(self.handle)
        buf = np.zeros(nbytes, dtype=np.uint8)
        _check(_lib.ns_checkpoint_save(self.handle, buf.ctypes.data_as(_P), nbytes), "ns_checkpoint_save")
        return buf

    def restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib.ns_checkpoint_load(self.handle, buf.ctypes.data_as(_P), buf.size), "ns_checkpoint_load")

    # ---- step-size proposer
    def mlp_set_weights(self, w):
        ns_mlp_set_weights(self.handle, w)

    def mlp_get_weights(self):
        out = np.zeros(NS_MLP_NWEIGHTS, dtype=np.float32)
        ns_mlp_get_weights(self.handle, out)
        return out

    def _f32(self, a):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(self.device).contiguous()

    def mlp_forward(self, x):
        xd = self._f32(x)
        n = xd.shape[0]
        y = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        self.torch.cuda.synchronize(self.device)
        ns_mlp_forward(self.handle, xd.data_ptr(), n, y.data_ptr())
        self.stream.synchronize()
        return y.cpu().numpy()

    def mlp_grad(self, x, t):
        xd, td = self._f32(x), self._f32(t)
        g = np.zeros(NS_MLP_NPARAM, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        self.torch.cuda.synchronize(self.device)
        ns_mlp_grad(self.handle, xd.data_ptr(), td.data_ptr(), xd.shape[0], g, loss)
        return float(loss[0]), g

    def mlp_train_batch(self, x, t, lr):
        xd, td = self._f32(x), self._f32(t)
        loss = np.zeros(1, dtype=np.float32)
        self.torch.cuda.synchronize(self.device)
        ns_mlp_train_batch(self.handle, xd.data_ptr(), td.data_ptr(), xd.shape[0], lr, loss)
        return float(loss[0])

    def mlp_reset_optimizer(self):
        ns_mlp_reset_optimizer(self.handle)

    def mlp_collect(self, enable=True):
        ns_mlp_collect(self.handle, enable)

    def mlp_rows(self, max_rows=65536):
        cnt = ns_mlp_rows(self.handle, None, None, 0)
        n = min(cnt, 65536, max_rows)
        x = np.zeros((n, 20), dtype=np.float32)
        y = np.zeros(n, dtype=np.float32)
        if n:
            ns_mlp_rows(self.handle, x, y, n)
        return x, y, cnt

    def mlp_push_rows(self, x, y):
        ns_mlp_push_rows(self.handle, x, y)

    def mlp_fit_stats(self):
        ns_mlp_fit_stats(self.handle)

    def mlp_train(self, iters, batch, lr, seed=0):
        loss = np.zeros(1, dtype=np.float32)
        ns_mlp_train(self.handle, iters, batch, lr, seed, loss)
        return float(loss[0])

    def time(self):
        t = np.zeros(self.batch)
        ns_get_time(self.handle, t)
        return t

    def set_time(self, t):
        ns_set_time(self.handle, np.broadcast_to(np.asarray(t, dtype=np.float64), (self.batch,)))

    def diagnostics(self):
        e = np.zeros(self.batch)
        eps = np.zeros(self.batch)
        sh = np.zeros(self.batch * 16)
        ns_diagnostics(self.handle, e, eps, sh)
        return e, eps, sh.reshape(self.batch, 16)

    def refresh_rhs(self):
        ns_refresh_rhs(self.handle)

    def autotune(self, reps=3):
        """Pick the fastest launch variant of each pass; returns
        (variants, ms[pass][variant])."""
        ms = np.zeros(NS_NTUNE * NS_TUNE_MAXV)
        ns_autotune(self.handle, reps, ms)
        return ns_tune_get(self.handle), ms.reshape(NS_NTUNE, NS_TUNE_MAXV)

    def tune(self, variants=None):
        if variants is not None:
            ns_tune_set(self.handle, variants)
        return ns_tune_get(self.handle)

    def profile_start(self):
        ns_profile_start(self.handle)

    def profile_mode(self, mode):
        """0 passes, 1 also every y/x/y launch, 2 whole evaluations only."""
        ns_profile_mode(self.handle, mode)

    def profile_stop(self):
        """{kernel name: (total ms, launches)} since profile_start."""
        out = NsKernelTimes()
        ns_profile_stop(self.handle, out)
        return {PROF_NAMES[i]: (out.ms[i], out.count[i]) for i in range(len(PROF_NAMES))}

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "handle", None):
            ns_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
