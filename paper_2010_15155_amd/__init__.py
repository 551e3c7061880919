"""MI355X kernel aggregated FMM: Python binding of ``libstkfmm.so``.

Argument marshalling only: every step of the evaluation pass runs in the
HIP library behind the C ABI declared in ``include/stkfmm.h``.  PyTorch
provides device memory (tensors) and the current HIP stream.  There is no
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

KERNELS = {"LapPGrad": 0, "Stokeslet": 1, "RPY": 2, "PVel": 3, "Traction": 4, "StokesRegVel": 5,
           "StokesRegVelOmega": 6, "LapPGradGrad": 7, "PVelGrad": 8, "PVelLaplacian": 9,
           "LapQPGradGrad": 10}
BCS = {"open": 0, "PX": 1, "PXY": 2, "PXYZ": 3, "wall": 4}
STATUS = {0: "OK", 1: "E_ARG", 2: "E_DOMAIN", 3: "E_UNSUPPORTED", 4: "E_NOMEM", 5: "E_DEVICE",
          6: "E_ACCURACY", 7: "E_STATE"}
STAGES = ["pack", "s2m", "upward", "m2l", "s2l", "downward", "l2t", "p2p", "combine", "m2l_gemm"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstkfmm.so")

# exported C symbols (kept in step with include/stkfmm.h)
SYMBOLS = ["stkfmm_setup", "stkfmm_set_points", "stkfmm_run", "stkfmm_evaluate", "stkfmm_direct",
           "stkfmm_kernel_dims", "stkfmm_set_option", "stkfmm_get_timings", "stkfmm_get_stats",
           "stkfmm_last_error", "stkfmm_destroy", "stkfmm_mlp_nparam", "stkfmm_mlp_workspace",
           "stkfmm_set_predictor", "stkfmm_get_learned", "stkfmm_get_leaf_features",
           "stkfmm_get_plan_work", "stkfmm_mlp_forward", "stkfmm_mlp_loss_grad", "stkfmm_mlp_adam",
           "stkfmm_get_tree", "stkfmm_direct_noalloc", "stkfmm_prepare_operators"]
ORDER_CLASSES = (6, 8, 10, 12)
CAP_CLASSES = (250, 500, 1000, 2000)

_lib = None


class StkfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = STATUS.get(status, status)


def lib():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libstkfmm.so is not built: run __graft_entry__.build() "
                           "or python paper_2010_15155_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.stkfmm_setup.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(cd), cd, ci, ctypes.c_uint]
    L.stkfmm_set_points.argtypes = [vp, ci, ci, i64, vp, i64, vp, i64, vp, ci, ci, vp]
    L.stkfmm_run.argtypes = [vp, vp, vp, vp, vp]
    L.stkfmm_evaluate.argtypes = [vp, ci, ci, i64, vp, vp, i64, vp, vp, i64, vp, vp, ci, ci, vp]
    L.stkfmm_direct.argtypes = [vp, ci, i64, vp, vp, i64, vp, vp, i64, vp, vp, vp]
    L.stkfmm_direct_noalloc.argtypes = [vp, ci, i64, vp, vp, i64, vp, vp, i64, vp, vp, vp]
    L.stkfmm_kernel_dims.argtypes = [ci, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.stkfmm_set_option.argtypes = [vp, ctypes.c_char_p, ctypes.c_char_p]
    L.stkfmm_get_timings.argtypes = [vp, ctypes.POINTER(cd), ctypes.POINTER(cd), ctypes.POINTER(cd)]
    L.stkfmm_get_stats.argtypes = [vp, ctypes.POINTER(i64)]
    L.stkfmm_get_tree.argtypes = [vp, ctypes.POINTER(i64), vp, vp, vp, vp]
    L.stkfmm_last_error.argtypes = [vp]
    L.stkfmm_last_error.restype = ctypes.c_char_p
    L.stkfmm_destroy.argtypes = [vp]
    L.stkfmm_destroy.restype = None
    L.stkfmm_mlp_nparam.argtypes = []
    L.stkfmm_mlp_workspace.argtypes = [i64]
    L.stkfmm_mlp_workspace.restype = i64
    L.stkfmm_set_predictor.argtypes = [vp, vp, ci]
    L.stkfmm_get_learned.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(cd)]
    L.stkfmm_get_leaf_features.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
    L.stkfmm_get_plan_work.argtypes = [vp, vp]
    L.stkfmm_prepare_operators.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_char_p, vp, vp]
    L.stkfmm_mlp_forward.argtypes = [vp, i64, vp, vp, vp, vp]
    L.stkfmm_mlp_loss_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.stkfmm_mlp_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp]
    _lib = L
    return L


def kernel_dims(kernel):
    k_sl, k_dl, k_t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    st = lib().stkfmm_kernel_dims(KERNELS[kernel], ctypes.byref(k_sl), ctypes.byref(k_dl), ctypes.byref(k_t))
    if st != 0:
        raise StkfmmError(st, "kernel_dims")
    return k_sl.value, k_dl.value, k_t.value


def prepare_operators(p, bc="open", svd_tol=1e-7, m2l_tol=0.0, cache_dir=None):
    """Build or load the host operator set of order p for boundary bc through
    the on-disk cache (stkfmm_prepare_operators; host only, no device).
    Returns (loaded, digest): loaded is True when the set came from cache_dir."""
    loaded, digest = ctypes.c_int(), ctypes.c_uint64()
    d = None if cache_dir is None else os.fsencode(cache_dir)
    st = lib().stkfmm_prepare_operators(int(p), BCS[bc], float(svd_tol), float(m2l_tol), d,
                                        ctypes.byref(loaded), ctypes.byref(digest))
    if st != 0:
        raise StkfmmError(st, "prepare_operators")
    return bool(loaded.value), int(digest.value)


def _ptr(t, n_cols, name, device=None, rows=None):
    """Device pointer and row count of a contiguous float64 CUDA tensor (or
    (None, 0)).  With `device` the tensor must live on cuda:device; with
    `rows` it must hold exactly that many rows (the library reads or writes
    every one of them)."""
    if t is None:
        if rows:
            raise ValueError("%s is required: the plan has %d of its points" % (name, rows))
        return None, 0
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 tensor on the GPU" % name)
    if device is not None and t.device.index != device:
        raise ValueError("%s is on %s, the context on cuda:%d" % (name, t.device, device))
    if n_cols and (t.dim() != 2 or t.shape[1] != n_cols) and not (n_cols == 1 and t.dim() == 1):
        raise ValueError("%s must have shape [n, %d]" % (name, n_cols))
    if rows is not None and t.shape[0] != rows:
        raise ValueError("%s has %d rows, the plan %d" % (name, t.shape[0], rows))
    return ctypes.c_void_p(t.data_ptr()), t.shape[0]


def _stream(device):
    """The current torch stream of cuda:device."""
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class FMM:
    """One library context (stkfmm_setup ... stkfmm_destroy)."""

    def __init__(self, origin=(0.0, 0.0, 0.0), box_len=1.0, device=0):
        self._h = ctypes.c_void_p()
        org = (ctypes.c_double * 3)(*origin)
        st = lib().stkfmm_setup(ctypes.byref(self._h), org, float(box_len), int(device), 0)
        if st != 0:
            raise StkfmmError(st, "stkfmm_setup")
        self.device = device
        self.kernel = None
        self.n_sl = self.n_dl = self.n_trg = 0

    def _check(self, st, what):
        if st != 0:
            raise StkfmmError(st, "%s: %s" % (what, lib().stkfmm_last_error(self._h).decode()))

    def close(self):
        if self._h:
            lib().stkfmm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key, value):
        self._check(lib().stkfmm_set_option(self._h, key.encode(), str(value).encode()), "set_option")

    def set_points(self, kernel, sl_xyz=None, dl_xyz=None, trg_xyz=None, p=10, leaf_cap=2000, bc="open"):
        s, ns = _ptr(sl_xyz, 3, "sl_xyz", self.device)
        d, nd = _ptr(dl_xyz, 3, "dl_xyz", self.device)
        t, nt = _ptr(trg_xyz, 3, "trg_xyz", self.device)
        self.kernel = None
        st = lib().stkfmm_set_points(self._h, KERNELS[kernel], BCS[bc], ns, s, nd, d, nt, t,
                                     int(p), int(leaf_cap), _stream(self.device))
        self._check(st, "set_points")
        self.kernel = kernel
        self.n_sl, self.n_dl, self.n_trg = ns, nd, nt

    def run(self, sl_val=None, dl_val=None, out=None):
        """Evaluation pass on the points of the last set_points: sl_val [n_sl, k_sl],
        dl_val [n_dl, k_dl] (row counts as planned), out [n_trg, k_trg] (allocated
        when None)."""
        import torch
        if self.kernel is None:
            raise RuntimeError("run before a successful set_points")
        k_sl, k_dl, k_t = kernel_dims(self.kernel)
        s, _ = _ptr(sl_val, k_sl, "sl_val", self.device, self.n_sl)
        d, _ = _ptr(dl_val, k_dl, "dl_val", self.device, self.n_dl)
        if out is None:
            out = torch.empty((self.n_trg, k_t), dtype=torch.float64, device="cuda:%d" % self.device)
        o, _ = _ptr(out, k_t, "trg_val", self.device, self.n_trg)
        self._check(lib().stkfmm_run(self._h, s, d, o, _stream(self.device)), "run")
        return out

    def evaluate(self, kernel, sl_xyz=None, sl_val=None, dl_xyz=None, dl_val=None, trg_xyz=None,
                 p=10, leaf_cap=2000, bc="open"):
        self.set_points(kernel, sl_xyz, dl_xyz, trg_xyz, p, leaf_cap, bc)
        return self.run(sl_val, dl_val)

    def direct(self, kernel, sl_xyz=None, sl_val=None, dl_xyz=None, dl_val=None, trg_xyz=None, out=None,
               noalloc=False):
        """FP64 direct sum on the GPU (error judge) into `out` [n_trg, k_trg] (allocated
        when None).  noalloc=True calls stkfmm_direct_noalloc, whose partial sums live
        in the library's static device scratch instead of memory it allocates."""
        import torch
        k_sl, k_dl, k_t = kernel_dims(kernel)
        s, ns = _ptr(sl_xyz, 3, "sl_xyz", self.device)
        sv, _ = _ptr(sl_val, k_sl, "sl_val", self.device, ns)
        d, nd = _ptr(dl_xyz, 3, "dl_xyz", self.device)
        dv, _ = _ptr(dl_val, k_dl, "dl_val", self.device, nd)
        t, nt = _ptr(trg_xyz, 3, "trg_xyz", self.device)
        if out is None:
            out = torch.empty((nt, k_t), dtype=torch.float64, device="cuda:%d" % self.device)
        o, _ = _ptr(out, k_t, "trg_val", self.device, nt)
        fn = lib().stkfmm_direct_noalloc if noalloc else lib().stkfmm_direct
        st = fn(self._h, KERNELS[kernel], ns, s, sv, nd, d, dv, nt, t, o, _stream(self.device))
        self._check(st, "direct_noalloc" if noalloc else "direct")
        return out

    def timings(self):
        tt, tr = ctypes.c_double(), ctypes.c_double()
        stg = (ctypes.c_double * 16)()
        self._check(lib().stkfmm_get_timings(self._h, ctypes.byref(tt), ctypes.byref(tr), stg), "timings")
        return {"t_tree_ms": tt.value, "t_run_ms": tr.value,
                "stages_ms": {k: stg[i] for i, k in enumerate(STAGES)}}

    def stats(self):
        a = (ctypes.c_int64 * 21)()
        self._check(lib().stkfmm_get_stats(self._h, a), "stats")
        names = ["boxes", "leaves", "depth", "u_pairs", "v_pairs", "w_pairs", "x_pairs", "M",
                 "n_trg", "n_sl", "n_dl", "u_entries", "p2p_pairs", "w_direct", "x_direct", "p2p_tasks",
                 "m2l_rank", "Mp", "pinv_rank", "p2p_lane_pairs", "p2p_exact_r"]
        return {n: int(a[i]) for i, n in enumerate(names)}

    def tree(self):
        """The octree and U/V/W/X lists of the current plan as NumPy arrays: box [n_box, 12]
        (level, anchor xyz, parent, is_leaf, SL/DL/target ranges), perm_sl/perm_dl/perm_trg
        (sorted position -> input index) and, per list, CSR offsets [n_box + 1] and entries
        [n, 4] (box, shift xyz)."""
        import numpy as np
        sz = (ctypes.c_int64 * 8)()
        self._check(lib().stkfmm_get_tree(self._h, sz, None, None, None, None), "get_tree")
        nb, nu, nv, nw, nx, ns, nd, nt = (int(v) for v in sz)
        box = np.zeros((nb, 12), dtype=np.int32)
        perm = np.zeros(ns + nd + nt, dtype=np.int32)
        off = np.zeros((4, nb + 1), dtype=np.int32)
        ent = np.zeros((nu + nv + nw + nx, 4), dtype=np.int32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(lib().stkfmm_get_tree(self._h, sz, ptr(box), ptr(perm), ptr(off), ptr(ent)), "get_tree")
        out = {"box": box, "perm_sl": perm[:ns], "perm_dl": perm[ns:ns + nd], "perm_trg": perm[ns + nd:]}
        e0 = 0
        for q, (name, n) in enumerate(zip("UVWX", (nu, nv, nw, nx))):
            out[name + "_off"] = off[q]
            out[name] = ent[e0:e0 + n]
            e0 += n
        return out

    # ---------------------------------------------------------------- learned mode
    def set_predictor(self, params):
        """Install predictor parameters (NumPy float32, stkfmm_mlp_nparam() values)."""
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().stkfmm_set_predictor(self._h, p.ctypes.data_as(ctypes.c_void_p), int(p.size)),
                    "set_predictor")

    def learned_info(self):
        info = (ctypes.c_int64 * 12)()
        err = ctypes.c_double()
        self._check(lib().stkfmm_get_learned(self._h, info, ctypes.byref(err)), "get_learned")
        return {"learned": bool(info[0]), "p": int(info[1]), "fell_back": bool(info[2]),
                "validated": bool(info[3]), "order_hist": [int(info[4 + k]) for k in range(4)],
                "cap_hist": [int(info[8 + k]) for k in range(4)], "sampled_err": err.value}

    def leaf_features(self):
        """(features [n_leaf, 12] float32, leaf index of every target [n_trg]) of the current tree."""
        import numpy as np
        n = ctypes.c_int64()
        self._check(lib().stkfmm_get_leaf_features(self._h, None, None, ctypes.byref(n)), "leaf_features")
        feat = np.zeros((n.value, 12), dtype=np.float32)
        lot = np.zeros(self.n_trg, dtype=np.int32)
        self._check(lib().stkfmm_get_leaf_features(self._h, feat.ctypes.data_as(ctypes.c_void_p),
                                                   lot.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)),
                    "leaf_features")
        return feat, lot

    def plan_work(self):
        """Work of the current plan per target [n_trg, 5] (user order): P2P lane pairs,
        P2P wave entries, M2L flops, surface evaluations, boxes."""
        import numpy as np
        n = self.stats()["n_trg"]
        out = np.zeros((n, 5))
        self._check(lib().stkfmm_get_plan_work(self._h, out.ctypes.data_as(ctypes.c_void_p)), "plan_work")
        return out


def mlp_nparam():
    return int(lib().stkfmm_mlp_nparam())


def _dev(t, dtype, name):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("%s must be a contiguous %s tensor on the GPU" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


def _work(batch, device):
    import torch
    return torch.empty(int(lib().stkfmm_mlp_workspace(int(batch))), dtype=torch.float32, device=device)


def mlp_forward(params, x):
    """Logits [batch, 8] of the predictor network (device tensors, float32)."""
    import torch
    out = torch.empty((x.shape[0], 8), dtype=torch.float32, device=x.device)
    w = _work(x.shape[0], x.device)
    st = lib().stkfmm_mlp_forward(_dev(params, torch.float32, "params"), int(x.shape[0]),
                                  _dev(x, torch.float32, "x"), _dev(out, torch.float32, "logits"),
                                  _dev(w, torch.float32, "work"), _stream(x.device.index))
    if st != 0:
        raise StkfmmError(st, "mlp_forward")
    return out


def mlp_loss_grad(params, x, labels):
    """(loss, gradient [nparam]) of the mean two-head cross-entropy."""
    import torch
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    w = _work(x.shape[0], x.device)
    st = lib().stkfmm_mlp_loss_grad(_dev(params, torch.float32, "params"), int(x.shape[0]),
                                    _dev(x, torch.float32, "x"), _dev(labels, torch.int32, "labels"),
                                    _dev(grad, torch.float32, "grad"), _dev(loss, torch.float32, "loss"),
                                    _dev(w, torch.float32, "work"), _stream(x.device.index))
    if st != 0:
        raise StkfmmError(st, "mlp_loss_grad")
    return loss, grad


def mlp_adam(params, grad, m, v, step, lr):
    """One Adam step in place on the device parameter vector."""
    import torch
    st = lib().stkfmm_mlp_adam(_dev(params, torch.float32, "params"), _dev(grad, torch.float32, "grad"),
                               _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"), int(step), float(lr),
                               _stream(params.device.index))
    if st != 0:
        raise StkfmmError(st, "mlp_adam")
