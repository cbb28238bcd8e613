"""ctypes binding of the C ABI in include/mr.h (argument marshalling only).

Every operation runs in the HIP library ``libmr.so`` built in this package
directory; importing this module without that library raises, there is no
fallback implementation.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmr.so")

MR_OK, MR_EINVAL, MR_ENOMEM, MR_ECAPACITY, MR_EHIP, MR_ESTATE, MR_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
MR_F64, MR_F32 = 0, 1
MR_VEL_CONST, MR_VEL_ROTATING, MR_VEL_SHEAR, MR_VEL_DIFFUSION = 0, 1, 2, 3
MR_IC_GAUSS_SUM, MR_IC_TANH_SHELL = 0, 1


class mr_config(C.Structure):
    _fields_ = [("nb", C.c_int32), ("wavelet_N", C.c_int32), ("wavelet_Nt", C.c_int32),
                ("fd_order", C.c_int32), ("level_min", C.c_int32), ("level_max", C.c_int32),
                ("prec", C.c_int32), ("detail_ext", C.c_int32), ("n_fields", C.c_int32),
                ("exec_mode", C.c_int32), ("eps_refine", C.c_double),
                ("eps_coarsen", C.c_double), ("max_blocks", C.c_int64)]


class mr_tuning(C.Structure):
    _fields_ = [("lds_refine", C.c_int32), ("lds_restrict", C.c_int32),
                ("lds_subst", C.c_int32), ("subst_threads", C.c_int32),
                ("reserved", C.c_int32 * 4)]


class mr_velocity(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("p", C.c_double * 8)]


class mr_ic(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("params", C.POINTER(C.c_double))]


class mr_adapt_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refined", C.c_int32), ("coarsened", C.c_int32),
                ("in_band", C.c_int32), ("n_blocks", C.c_int64)]


class MRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mr error %d: %s" % (code, msg))
        self.code = code


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmr.so is not built: run __graft_entry__.build() "
                          "(paper_2112_07537_amd/build_lib.py)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "mr_grid_create": [C.POINTER(mr_config), P, P, C.c_size_t, C.POINTER(P)],
        "mr_pool_bytes": [C.POINTER(mr_config), C.POINTER(C.c_size_t)],
        "mr_grid_destroy": [P],
        "mr_set_tree": [P, C.c_int64, P, P],
        "mr_sample_ic": [P, C.c_int32, C.POINTER(mr_ic)],
        "mr_init_ic": [P, C.c_int32, C.POINTER(mr_ic), C.c_int32, C.POINTER(mr_adapt_stats)],
        "mr_ghost": [P, C.c_int32, C.c_int32],
        "mr_ghost_get": [P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, P, C.c_size_t],
        "mr_details": [P, C.c_int32, P, C.c_int32],
        "mr_details_noalloc": [P, C.c_int32, P],
        "mr_adapt": [P, C.c_int32, C.c_int32, C.POINTER(mr_adapt_stats)],
        "mr_rk3_step": [P, C.c_int32, C.c_double, C.POINTER(mr_velocity)],
        "mr_stage": [P, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                     C.c_double, C.POINTER(mr_velocity)],
        "mr_set_thresholds": [P, C.c_double, C.c_double],
        "mr_ic_error": [P, C.c_int32, C.POINTER(mr_ic), P],
        "mr_adapt_flags": [P, P, C.POINTER(mr_adapt_stats)],
        "mr_set_tuning": [P, C.POINTER(mr_tuning)],
        "mr_get_tuning": [P, C.POINTER(mr_tuning)],
        "mr_device_arch": [C.c_char_p, C.c_size_t],
        "mr_details_rk3_step": [P, C.c_int32, C.c_double, C.POINTER(mr_velocity), P, C.c_int32],
        "mr_cfl_dt": [P, C.POINTER(mr_velocity), C.c_double, C.POINTER(C.c_double)],
        "mr_block_meta": [P, C.c_int64, C.POINTER(C.c_int64), P, P],
        "mr_field_get": [P, C.c_int32, P, C.c_size_t],
        "mr_field_set": [P, C.c_int32, P, C.c_size_t],
        "mr_field_ptr": [P, C.c_int32, C.POINTER(P)],
        "mr_moments": [P, C.c_int32, P],
        "mr_prof_enable": [P, C.c_int32],
        "mr_prof_read": [P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                         C.POINTER(C.c_int64)],
        "mr_tree_stats": [P, P],
        "mr_sync": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int32
    lib.mr_last_error.argtypes = []
    lib.mr_last_error.restype = C.c_char_p
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _check(code):
    if code != MR_OK:
        raise MRError(code, lib().mr_last_error().decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def device_arch():
    """mr_device_arch: the current HIP device's architecture name."""
    buf = C.create_string_buffer(64)
    _check(lib().mr_device_arch(buf, 64))
    return buf.value.decode()


def velocity(kind, *p):
    v = mr_velocity()
    v.kind = {"const": MR_VEL_CONST, "rotating": MR_VEL_ROTATING,
              "shear": MR_VEL_SHEAR, "diffusion": MR_VEL_DIFFUSION}.get(kind, kind)
    for i, x in enumerate(p):
        v.p[i] = float(x)
    return v


def make_config(nb, N, Nt, fd_order=4, level_min=0, level_max=12, prec="f64", eps_refine=1e-2,
                eps_coarsen=1e-4, detail_ext=1, n_fields=1, exec_mode=0, max_blocks=1 << 16):
    return mr_config(nb, N, Nt, fd_order, level_min, level_max,
                     MR_F32 if prec in ("f32", MR_F32) else MR_F64, detail_ext, n_fields,
                     exec_mode, eps_refine, eps_coarsen, max_blocks)


def pool_bytes(**kw):
    """Bytes a caller-owned pool must hold for the configuration (mr_pool_bytes)."""
    n = C.c_size_t()
    _check(lib().mr_pool_bytes(C.byref(make_config(**kw)), C.byref(n)))
    return n.value


class Grid:
    """Owning handle of an ``mr_grid``; methods map one-to-one to the C ABI."""

    def __init__(self, nb, N, Nt, fd_order=4, level_min=0, level_max=12, prec="f64",
                 eps_refine=1e-2, eps_coarsen=1e-4, detail_ext=1, n_fields=1,
                 exec_mode=0, max_blocks=1 << 16, stream=None, pool=None, pool_bytes=0):
        """``pool``: device address of caller-owned memory (e.g. the data_ptr()
        of a torch uint8 CUDA tensor, which the caller keeps alive) holding
        ``pool_bytes`` >= pool_bytes(cfg) for the field buffers."""
        c = make_config(nb, N, Nt, fd_order, level_min, level_max, prec, eps_refine,
                        eps_coarsen, detail_ext, n_fields, exec_mode, max_blocks)
        self.cfg = c
        self.dtype = np.float32 if c.prec == MR_F32 else np.float64
        self.nb = nb
        h = C.c_void_p()
        _check(lib().mr_grid_create(C.byref(c), C.c_void_p(stream), C.c_void_p(pool),
                                    C.c_size_t(pool_bytes), C.byref(h)))
        self.warning = lib().mr_last_error().decode()
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mr_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tree
    def set_tree(self, keys):
        keys = np.asarray(keys, dtype=np.int32).reshape(-1, 4)
        lev = np.ascontiguousarray(keys[:, 0])
        ijk = np.ascontiguousarray(keys[:, 1:4])
        _check(lib().mr_set_tree(self._h, len(keys), _ptr(lev), _ptr(ijk)))

    def block_meta(self):
        n = C.c_int64()
        _check(lib().mr_block_meta(self._h, 0, C.byref(n), None, None))
        lev = np.zeros(n.value, np.int32)
        ijk = np.zeros((n.value, 3), np.int32)
        _check(lib().mr_block_meta(self._h, n.value, C.byref(n), _ptr(lev), _ptr(ijk)))
        return np.concatenate([lev[:, None], ijk], axis=1)

    def n_blocks(self):
        n = C.c_int64()
        _check(lib().mr_block_meta(self._h, 0, C.byref(n), None, None))
        return n.value

    # -- fields
    def field_get(self, field=0):
        n = self.n_blocks()
        a = np.empty(n * self.nb ** 3, self.dtype)
        _check(lib().mr_field_get(self._h, field, _ptr(a), a.nbytes))
        return a.reshape(n, self.nb, self.nb, self.nb)

    def field_set(self, data, field=0):
        a = np.ascontiguousarray(data, dtype=self.dtype)
        _check(lib().mr_field_set(self._h, field, _ptr(a), a.nbytes))

    def field_ptr(self, field=0):
        p = C.c_void_p()
        _check(lib().mr_field_ptr(self._h, field, C.byref(p)))
        return p.value

    @staticmethod
    def _ic(kind, params):
        par = np.ascontiguousarray(params, dtype=np.float64).ravel()
        ic = mr_ic()
        if kind == "gauss":
            ic.kind, ic.n = MR_IC_GAUSS_SUM, len(par) // 5
        else:
            ic.kind, ic.n = MR_IC_TANH_SHELL, 1
        ic.params = par.ctypes.data_as(C.POINTER(C.c_double))
        return ic, par

    def sample_ic(self, kind, params, field=0):
        ic, keep = self._ic(kind, params)
        _check(lib().mr_sample_ic(self._h, field, C.byref(ic)))

    def init_ic(self, kind, params, field=0, max_iter=64):
        ic, keep = self._ic(kind, params)
        st = mr_adapt_stats()
        _check(lib().mr_init_ic(self._h, field, C.byref(ic), max_iter, C.byref(st)))
        return st

    # -- hot path
    def ghost(self, field=0, depth=0):
        _check(lib().mr_ghost(self._h, field, depth))

    def ghost_get(self, depth, b0=0, nblk=None, field=0):
        if nblk is None:
            nblk = self.n_blocks() - b0
        e = self.nb + 2 * depth
        a = np.empty(nblk * e ** 3, self.dtype)
        _check(lib().mr_ghost_get(self._h, field, depth, b0, nblk, _ptr(a), a.nbytes))
        return a.reshape(nblk, e, e, e)

    def details(self, field=0):
        n = self.n_blocks()
        a = np.empty(n, np.float64)
        _check(lib().mr_details(self._h, field, _ptr(a), 0))
        return a

    def stage(self, y, un, out, a_un, b, c_y, dt, vel):
        """mr_stage: out = a_un*un + b*(c_y*y + dt*L(y)) after y's ghost fill."""
        _check(lib().mr_stage(self._h, y, un, out, a_un, b, c_y, dt, C.byref(vel)))

    def rhs(self, y, out, vel):
        """L(y) into field `out` (mr_stage with a_un = 0, b = 1, c_y = 0, dt = 1)."""
        self.stage(y, y, out, 0.0, 1.0, 0.0, 1.0, vel)

    TUNING_KEYS = ("lds_refine", "lds_restrict", "lds_subst", "subst_threads")

    def set_tuning(self, **kw):
        """mr_set_tuning: launch-shape knobs (mr_tuning fields; omitted = keep)."""
        t = mr_tuning()
        for k, v in kw.items():
            if k not in self.TUNING_KEYS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(lib().mr_set_tuning(self._h, C.byref(t)))

    def get_tuning(self):
        t = mr_tuning()
        _check(lib().mr_get_tuning(self._h, C.byref(t)))
        return {k: int(getattr(t, k)) for k in self.TUNING_KEYS}

    def set_thresholds(self, eps_refine, eps_coarsen):
        _check(lib().mr_set_thresholds(self._h, eps_refine, eps_coarsen))

    def details_noalloc(self, dev_norms, field=0):
        """mr_details_noalloc: norms into caller device memory (address)."""
        _check(lib().mr_details_noalloc(self._h, field, C.c_void_p(dev_norms)))

    def details_async(self, dev_ptr=None, field=0):
        _check(lib().mr_details(self._h, field, C.c_void_p(dev_ptr), 1))

    def adapt(self, field=0, max_iter=64):
        st = mr_adapt_stats()
        _check(lib().mr_adapt(self._h, field, max_iter, C.byref(st)))
        return st

    def adapt_flags(self, flags):
        """mr_adapt_flags: one adaptation with caller block statuses (+1/0/-1)."""
        f = np.ascontiguousarray(flags, dtype=np.int8)
        if f.shape != (self.n_blocks(),):
            raise ValueError("one status per block")
        st = mr_adapt_stats()
        _check(lib().mr_adapt_flags(self._h, f.ctypes.data_as(C.c_void_p), C.byref(st)))
        return st

    def rk3_step(self, dt, vel, field=0):
        _check(lib().mr_rk3_step(self._h, field, dt, C.byref(vel)))

    def details_rk3_step(self, dt, vel, field=0):
        """Detail norms of the field, then one RK3 step that reuses their
        ghosts for its first stage; returns the norms (before the step)."""
        n = self.n_blocks()
        a = np.empty(n, np.float64)
        _check(lib().mr_details_rk3_step(self._h, field, dt, C.byref(vel), _ptr(a), 0))
        return a

    def details_rk3_step_async(self, dt, vel, dev_ptr=None, field=0):
        _check(lib().mr_details_rk3_step(self._h, field, dt, C.byref(vel), C.c_void_p(dev_ptr), 1))

    def cfl_dt(self, vel, cfl):
        dt = C.c_double()
        _check(lib().mr_cfl_dt(self._h, C.byref(vel), cfl, C.byref(dt)))
        return dt.value

    def moments(self, field=0):
        a = np.zeros(4, np.float64)
        _check(lib().mr_moments(self._h, field, _ptr(a)))
        return a

    def ic_error(self, kind, params, field=0):
        """mr_ic_error: (max |phi - f|, L2 norm of phi - f) over the leaves."""
        ic, par = self._ic(kind, params)
        a = np.zeros(2, np.float64)
        _check(lib().mr_ic_error(self._h, field, C.byref(ic), _ptr(a)))
        return float(a[0]), float(a[1])

    def prof_enable(self, on=True):
        _check(lib().mr_prof_enable(self._h, int(on)))

    def prof_read(self, kernel):
        ms = C.c_double()
        n = C.c_int64()
        pts = C.c_int64()
        _check(lib().mr_prof_read(self._h, kernel.encode(), C.byref(ms), C.byref(n), C.byref(pts)))
        return ms.value, n.value, pts.value

    def sync(self):
        _check(lib().mr_sync(self._h))

    def tree_stats(self):
        a = np.zeros(22, np.int64)
        _check(lib().mr_tree_stats(self._h, _ptr(a)))
        return a
