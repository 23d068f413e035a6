"""ctypes binding of libscasm.so: argument marshalling only; every step of the
assembly and of the iteration phase runs in the library (host planner and
HIP kernels).  Loading fails loudly when the library is missing."""
import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscasm.so")

SC_OK, SC_ERR_INVALID_ARG, SC_ERR_NOT_SPD, SC_ERR_OOM, SC_ERR_DEVICE, SC_ERR_UNSUPPORTED, SC_ERR_STATE = range(7)
SC_PREC_FP64, SC_PREC_MIXED = 0, 1
STATUS_NAMES = {0: "SC_OK", 1: "SC_ERR_INVALID_ARG", 2: "SC_ERR_NOT_SPD", 3: "SC_ERR_OOM",
                4: "SC_ERR_DEVICE", 5: "SC_ERR_UNSUPPORTED", 6: "SC_ERR_STATE"}

EXPORTED = ["sc_plan_create", "sc_factor", "sc_assemble", "sc_apply", "sc_apply_implicit",
            "sc_get_F", "sc_query", "sc_plan_stats", "sc_plan_destroy", "sc_host_analyze",
            "sc_host_tile_visits", "sc_set_timing", "sc_kernel_times", "sc_pcpg", "sc_autotune", "sc_autotune_classes", "sc_apply_noalloc", "sc_preprocess", "sc_query_selection",
            "sc_last_error"]


class ScasmError(RuntimeError):
    def __init__(self, status, message, failed_sub=None, failed_col=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message
        self.failed_sub = failed_sub
        self.failed_col = failed_col


class SubdomainDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("kreg_rowptr", ctypes.c_void_p), ("kreg_col", ctypes.c_void_p),
                ("m", ctypes.c_int32), ("bt_dof", ctypes.c_void_p), ("bt_sign", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("coords", ctypes.c_void_p), ("dim", ctypes.c_int32),
                ("dofs_per_node", ctypes.c_int32)]


class TuneClass(ctypes.Structure):
    _fields_ = [("n_lo", ctypes.c_int32), ("n_hi", ctypes.c_int32), ("panel_width", ctypes.c_int32),
                ("block_split", ctypes.c_int32), ("syrk_kind", ctypes.c_int32), ("ms_per_sub", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("disable_staircase", ctypes.c_int32),
                ("panel_width", ctypes.c_int32), ("relax_width", ctypes.c_int32),
                ("leaf_nodes", ctypes.c_int32), ("n_threads", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("assembly_kernels", ctypes.c_int32),
                ("disable_reach", ctypes.c_int32), ("block_split", ctypes.c_int32), ("select_iters", ctypes.c_int32),
                ("select_model", ctypes.c_float * 3),
                ("arena_cap_bytes", ctypes.c_int64), ("tune_classes", ctypes.POINTER(TuneClass)),
                ("ntune_classes", ctypes.c_int32), ("lower_only_csr", ctypes.c_int32), ("syrk_kind", ctypes.c_int32),
                ("disable_pair_merge", ctypes.c_int32)]


class HostInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("nnzL", ctypes.c_int64),
                ("nnzL_stored", ctypes.c_int64), ("nsuper", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("max_width", ctypes.c_int64), ("sum_below", ctypes.c_int64),
                ("trsm_useful", ctypes.c_double), ("syrk_useful", ctypes.c_double),
                ("trsm_dense", ctypes.c_double), ("syrk_dense", ctypes.c_double),
                ("factor_flops", ctypes.c_double), ("trsm_visits", ctypes.c_int64),
                ("stair_visits", ctypes.c_int64), ("trsm_reach", ctypes.c_double),
                ("syrk_reach", ctypes.c_double), ("t_asm_ms", ctypes.c_double), ("t_expl_ms", ctypes.c_double),
                ("t_impl_ms", ctypes.c_double), ("n_star", ctypes.c_double),
                ("merge_pairs", ctypes.c_int64), ("merged_rows", ctypes.c_int64),
                ("pruned_updates", ctypes.c_int64)]


_lib = None


def load():
    """The shared library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2509_21037_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64p, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        lib.sc_plan_create.argtypes = [ctypes.POINTER(SubdomainDesc), i32, ctypes.POINTER(Options), vp,
                                       ctypes.POINTER(vp)]
        lib.sc_factor.argtypes = [vp, ctypes.POINTER(vp), vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.sc_assemble.argtypes = [vp, vp]
        lib.sc_preprocess.argtypes = [vp, ctypes.POINTER(vp), vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.sc_apply.argtypes = [vp, vp, vp, vp]
        lib.sc_apply_implicit.argtypes = [vp, vp, vp, vp]
        lib.sc_apply_noalloc.argtypes = [vp, vp, vp, vp]
        lib.sc_get_F.argtypes = [vp, i32, vp, i32, i32, vp]
        lib.sc_query.argtypes = [vp, i32, i64p, i64p, i64p, i64p, dp]
        lib.sc_plan_stats.argtypes = [vp, ctypes.POINTER(i32), i64p, dp, dp, dp, dp, dp, dp, i64p]
        lib.sc_plan_destroy.argtypes = [vp]
        lib.sc_host_analyze.argtypes = [ctypes.POINTER(SubdomainDesc), ctypes.POINTER(Options), vp, vp, vp,
                                         vp, vp, ctypes.POINTER(HostInfo), ctypes.POINTER(i32)]
        lib.sc_host_tile_visits.argtypes = [ctypes.POINTER(SubdomainDesc), ctypes.POINTER(Options), vp, vp, vp,
                                             vp, ctypes.c_int64, vp]
        lib.sc_pcpg.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), vp, vp, i32, vp, vp]
        lib.sc_autotune.argtypes = [ctypes.POINTER(SubdomainDesc), i32, ctypes.POINTER(Options),
                                    ctypes.POINTER(vp), ctypes.POINTER(i32), i32, i32, i32, vp,
                                    ctypes.POINTER(i32), dp]
        lib.sc_autotune_classes.argtypes = [ctypes.POINTER(SubdomainDesc), i32, ctypes.POINTER(Options),
                                            ctypes.POINTER(vp), i32, i32, ctypes.c_char_p, vp,
                                            ctypes.POINTER(TuneClass), i32, ctypes.POINTER(i32)]
        lib.sc_query_selection.argtypes = [vp, i32, ctypes.POINTER(i32), dp, dp, dp, dp]
        lib.sc_set_timing.argtypes = [vp, i32]
        lib.sc_kernel_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), i32]
        lib.sc_last_error.argtypes = []
        lib.sc_last_error.restype = ctypes.c_char_p
        for name in EXPORTED[:-1]:
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(status, **kw):
    if status != SC_OK:
        msg = load().sc_last_error().decode(errors="replace")
        raise ScasmError(status, msg, **kw)


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _fill_desc(d, s, keep, use_coords=True):
    rowptr = np.ascontiguousarray(s.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(s.col, dtype=np.int32)
    dof = np.ascontiguousarray(s.dof, dtype=np.int32)
    sign = np.ascontiguousarray(s.sign, dtype=np.int8)
    coords = getattr(s, "coords", None) if use_coords else None
    perm = getattr(s, "perm", None)
    d.n = int(s.n)
    d.kreg_rowptr = rowptr.ctypes.data
    d.kreg_col = col.ctypes.data
    d.m = int(dof.shape[0])
    d.bt_dof = dof.ctypes.data if dof.size else None
    d.bt_sign = sign.ctypes.data if sign.size else None
    keep += [rowptr, col, dof, sign]
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        d.perm = perm.ctypes.data
        keep.append(perm)
    if coords is not None:
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        d.coords = coords.ctypes.data
        d.dim = int(coords.shape[1])
        keep.append(coords)
    d.dofs_per_node = int(getattr(s, "dofs_per_node", 1))


ASSEMBLY_KERNELS = {"default": 0, "overlap": 1, "separate": 2}


def check_dual_tensor(t, length: int, device_index: int, name: str):
    """Raises ScasmError(SC_ERR_INVALID_ARG) unless `t` is a contiguous FP64
    tensor on HIP device `device_index` with at least `length` elements: the
    library reads and writes `length` doubles through its data pointer."""
    import torch
    bad = None
    if not isinstance(t, torch.Tensor):
        bad = f"{name} must be a torch.Tensor, got {type(t).__name__}"
    elif t.dtype != torch.float64:
        bad = f"{name} must be float64, got {t.dtype}"
    elif not t.is_contiguous():
        bad = f"{name} must be contiguous"
    elif t.numel() < length:
        bad = f"{name} has {t.numel()} elements, the plan's dual vectors have {length}"
    elif not t.is_cuda:
        bad = f"{name} must be a device tensor, got one on {t.device}"
    elif t.device.index != device_index:
        bad = f"{name} is on device {t.device.index}, the plan on device {device_index}"
    if bad is not None:
        raise ScasmError(SC_ERR_INVALID_ARG, bad)


BLOCK_SPLIT = {"uniform": 0, "etree": 1}


def _options(precision="fp64", staircase=True, panel_width=0, relax_width=0, leaf_nodes=0, n_threads=0,
             use_graph=False, assembly="default", reach=True, block_split="uniform", arena_cap_bytes=0,
             tune_classes=None, select_iters=0, select_model=(0.0, 0.0, 0.0), lower_only_csr=False, syrk_kind=0,
             pair_merge=True):
    opt = Options()
    opt.lower_only_csr = 1 if lower_only_csr else 0
    opt.syrk_kind = int(syrk_kind)
    opt.disable_pair_merge = 0 if pair_merge else 1
    opt.arena_cap_bytes = int(arena_cap_bytes)
    opt.select_iters = int(select_iters)
    for k in range(3):
        opt.select_model[k] = float(select_model[k])
    if tune_classes:
        arr = (TuneClass * len(tune_classes))()
        for k, c in enumerate(tune_classes):
            d = c.as_dict() if isinstance(c, TuneClass) else c
            arr[k] = TuneClass(int(d["n_lo"]), int(d["n_hi"]), int(d.get("panel_width", 0)),
                               int(d.get("block_split", -1)), int(d.get("syrk_kind", 0)),
                               float(d.get("ms_per_sub", 0.0)))
        opt.tune_classes = ctypes.cast(arr, ctypes.POINTER(TuneClass))
        opt.ntune_classes = len(tune_classes)
        opt._keep = arr                       # the array lives as long as the options
    opt.disable_reach = 0 if reach else 1
    opt.block_split = BLOCK_SPLIT[block_split] if isinstance(block_split, str) else int(block_split)
    opt.use_graph = 1 if use_graph else 0
    opt.assembly_kernels = ASSEMBLY_KERNELS[assembly] if isinstance(assembly, str) else int(assembly)
    opt.precision = {"fp64": SC_PREC_FP64, "mixed": SC_PREC_MIXED}.get(precision, precision) \
        if isinstance(precision, str) else int(precision)
    opt.disable_staircase = 0 if staircase else 1
    opt.panel_width = panel_width
    opt.relax_width = relax_width
    opt.leaf_nodes = leaf_nodes
    opt.n_threads = n_threads
    return opt


def host_analyze(s, values=True, want_L=False, use_coords=True, **opts):
    """Host-only planner run for one subdomain (no device needed).  Returns a
    dict with perm, pivots (sorted), pi (sorted -> original), statistics and,
    when want_L, the dense factor L (row-major, n <= 4096)."""
    lib = load()
    keep = []
    d = SubdomainDesc()
    _fill_desc(d, s, keep, use_coords)
    opt = _options(**opts)
    n, m = int(s.n), int(np.asarray(s.dof).shape[0])
    perm = np.zeros(n, dtype=np.int32)
    piv = np.zeros(max(1, m), dtype=np.int32)
    pi = np.zeros(max(1, m), dtype=np.int32)
    L = np.zeros((n, n)) if want_L else None
    vals = np.ascontiguousarray(s.val, dtype=np.float64) if values else None
    info = HostInfo()
    fc = ctypes.c_int32(-1)
    st = lib.sc_host_analyze(ctypes.byref(d), ctypes.byref(opt), vals.ctypes.data if vals is not None else None,
                             perm.ctypes.data, L.ctypes.data if L is not None else None, piv.ctypes.data,
                             pi.ctypes.data, ctypes.byref(info), ctypes.byref(fc))
    if st != SC_OK:
        _check(st, failed_col=fc.value)
    out = {f: getattr(info, f) for f, _ in HostInfo._fields_}
    out.update(perm=perm, piv=piv[:m], pi=pi[:m], L=L)
    return out


def host_tile_visits(s, use_coords=True, with_masks=False, **opts):
    """Factor blocks the TRSM visits per 64-column X tile (sc_host_tile_visits):
    returns (block_row0 [nblocks + 1], visit_ptr [ntiles + 1], visit), and with
    with_masks the 16-row step masks [ntiles, words] (uint64) as a fourth item."""
    lib = load()
    keep = []
    d = SubdomainDesc()
    _fill_desc(d, s, keep, use_coords)
    opt = _options(**opts)
    counts = np.zeros(4, dtype=np.int64)
    _check(lib.sc_host_tile_visits(ctypes.byref(d), ctypes.byref(opt), counts.ctypes.data, None, None, None, 0,
                                   None))
    nb, nt, tot, nw = (int(c) for c in counts)
    row0 = np.zeros(nb + 1, dtype=np.int32)
    ptr = np.zeros(nt + 1, dtype=np.int64)
    visit = np.zeros(max(1, tot), dtype=np.int32)
    masks = np.zeros((max(1, nt), max(1, nw)), dtype=np.uint64)
    _check(lib.sc_host_tile_visits(ctypes.byref(d), ctypes.byref(opt), counts.ctypes.data, row0.ctypes.data,
                                   ptr.ctypes.data, visit.ctypes.data, tot, masks.ctypes.data))
    if with_masks:
        return row0, ptr, visit[:tot], masks[:nt, :nw]
    return row0, ptr, visit[:tot]


def autotune(subdomains, candidates=(32, 48, 64), sample=64, reps=3, use_coords=True, stream=None, **opts):
    """Fastest factor block width for this batch (sc_autotune): returns
    (best_width, {width: mean ms per assembly of the sample})."""
    lib = load()
    keep = []
    subs = list(subdomains)
    descs = (SubdomainDesc * len(subs))()
    for i, s in enumerate(subs):
        _fill_desc(descs[i], s, keep, use_coords)
    arrs = [np.ascontiguousarray(s.val, dtype=np.float64) for s in subs]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    cands = (ctypes.c_int32 * len(candidates))(*candidates)
    times = (ctypes.c_double * len(candidates))()
    best = ctypes.c_int32(0)
    opt = _options(**opts)
    _check(lib.sc_autotune(descs, len(subs), ctypes.byref(opt), ptrs, cands, len(candidates), int(sample),
                           int(reps), _stream_handle(stream), ctypes.byref(best), times))
    return best.value, {c: times[i] for i, c in enumerate(candidates)}


def autotune_classes(subdomains, sample=8, reps=2, cache_path=None, use_coords=True, stream=None, **opts):
    """Per-size-class settings (sc_autotune_classes): returns a list of dicts
    (n_lo, n_hi, panel_width, block_split, syrk_kind, ms_per_sub), to pass as
    Plan(..., tune_classes=...)."""
    lib = load()
    keep = []
    subs = list(subdomains)
    descs = (SubdomainDesc * len(subs))()
    for i, s in enumerate(subs):
        _fill_desc(descs[i], s, keep, use_coords)
    arrs = [np.ascontiguousarray(s.val, dtype=np.float64) for s in subs]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    out = (TuneClass * 21)()
    nc = ctypes.c_int32(0)
    opt = _options(**opts)
    _check(lib.sc_autotune_classes(descs, len(subs), ctypes.byref(opt), ptrs, int(sample), int(reps),
                                   cache_path.encode() if cache_path else None, _stream_handle(stream), out, 21,
                                   ctypes.byref(nc)))
    return [out[k].as_dict() for k in range(nc.value)]


class Plan:
    """A batch of subdomains (objects with n, rowptr, col, val, dof, sign and
    optional coords, dim, dofs_per_node, perm attributes)."""

    def __init__(self, subdomains: Sequence, precision: str = "fp64", staircase: bool = True,
                 panel_width: int = 0, relax_width: int = 0, leaf_nodes: int = 0, n_threads: int = 0,
                 use_coords: bool = True, use_graph: bool = False, assembly: str = "default", reach: bool = True,
                 block_split: str = "uniform", arena_cap_bytes: int = 0, tune_classes=None, select_iters: int = 0,
                 select_model=(0.0, 0.0, 0.0), lower_only_csr: bool = False, syrk_kind: int = 0,
                 pair_merge: bool = True, stream=None):
        lib = load()
        self._lib = lib
        self._h = ctypes.c_void_p(0)
        self.subdomains = list(subdomains)
        self.precision = precision
        keep = []
        descs = (SubdomainDesc * max(1, len(self.subdomains)))()
        for i, s in enumerate(self.subdomains):
            _fill_desc(descs[i], s, keep, use_coords)
        opt = _options(precision, staircase, panel_width, relax_width, leaf_nodes, n_threads, use_graph, assembly,
                       reach, block_split, arena_cap_bytes, tune_classes, select_iters, select_model,
                       lower_only_csr, syrk_kind, pair_merge)
        _check(lib.sc_plan_create(descs, len(self.subdomains), ctypes.byref(opt), _stream_handle(stream),
                                  ctypes.byref(self._h)))
        del keep
        import torch
        self.device_index = torch.cuda.current_device()
        self.dual_total = self.stats()["dual_total"]

    def _dual(self, t, name):
        check_dual_tensor(t, self.dual_total, self.device_index, name)
        return ctypes.c_void_p(t.data_ptr())

    # ---------------------------------------------------------------- stages
    def factor(self, kvals: Optional[List[np.ndarray]] = None, stream=None):
        if kvals is None:
            kvals = [s.val for s in self.subdomains]
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in kvals]
        ptrs = (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
        fs, fc = ctypes.c_int32(-1), ctypes.c_int32(-1)
        st = self._lib.sc_factor(self._h, ptrs, _stream_handle(stream), ctypes.byref(fs), ctypes.byref(fc))
        if st != SC_OK:
            _check(st, failed_sub=fs.value, failed_col=fc.value)
        # the upload is asynchronous and reads pinned memory owned by the plan
        return self

    def preprocess(self, kvals: Optional[List[np.ndarray]] = None, stream=None):
        """Factorisation and assembly in one pipelined call (host factorisation
        of later subdomain groups overlapped with the GPU assembly of earlier
        ones); F as after factor() + assemble()."""
        if kvals is None:
            kvals = [s.val for s in self.subdomains]
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in kvals]
        ptrs = (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
        fs, fc = ctypes.c_int32(-1), ctypes.c_int32(-1)
        st = self._lib.sc_preprocess(self._h, ptrs, _stream_handle(stream), ctypes.byref(fs), ctypes.byref(fc))
        if st != SC_OK:
            _check(st, failed_sub=fs.value, failed_col=fc.value)
        return self

    def assemble(self, stream=None):
        _check(self._lib.sc_assemble(self._h, _stream_handle(stream)))
        return self

    def apply(self, p, q, stream=None):
        """q = F p on device FP64 tensors of length dual_total."""
        pp, qp = self._dual(p, "p"), self._dual(q, "q")
        _check(self._lib.sc_apply(self._h, pp, qp, _stream_handle(stream)))
        return q

    def apply_noalloc(self, p, q, stream=None):
        """q = F p like apply(), through the entry point that allocates
        nothing (partial sums in the library's fixed per-GPU array)."""
        pp, qp = self._dual(p, "p"), self._dual(q, "q")
        _check(self._lib.sc_apply_noalloc(self._h, pp, qp, _stream_handle(stream)))
        return q

    def apply_implicit(self, p, q, stream=None):
        pp, qp = self._dual(p, "p"), self._dual(q, "q")
        _check(self._lib.sc_apply_implicit(self._h, pp, qp, _stream_handle(stream)))
        return q

    def pcpg(self, d, lam, iters: int, R_list=None, history: bool = False, stream=None):
        """Projected CG on every subdomain's dual problem; d, lam: device FP64
        tensors of length dual_total.  R_list: per-subdomain kernel bases
        (n_i x k_i); default: the subdomains' `R` attributes.  Returns the
        ||w_k|| history ((iters + 1) x nsub) when `history`."""
        if R_list is None:
            R_list = [s.R for s in self.subdomains]
        Rs = [np.asfortranarray(np.asarray(R, dtype=np.float64)) for R in R_list]
        ks = (ctypes.c_int32 * max(1, len(Rs)))(*[R.shape[1] for R in Rs])
        ptrs = (ctypes.c_void_p * max(1, len(Rs)))(*[R.ctypes.data for R in Rs])
        hist = np.zeros((iters + 1, len(Rs))) if history else None
        if len(Rs) != len(self.subdomains):
            raise ScasmError(SC_ERR_INVALID_ARG, f"{len(Rs)} kernel bases for {len(self.subdomains)} subdomains")
        for i, (R, s) in enumerate(zip(Rs, self.subdomains)):
            if R.ndim != 2 or R.shape[0] != int(s.n):
                raise ScasmError(SC_ERR_INVALID_ARG, f"R[{i}] must be n_i x k_i, got {R.shape}")
        dp, lp = self._dual(d, "d"), self._dual(lam, "lambda")
        _check(self._lib.sc_pcpg(self._h, ptrs, ks, dp, lp,
                                 int(iters), hist.ctypes.data if hist is not None else None,
                                 _stream_handle(stream)))
        return hist

    # ---------------------------------------------------------------- queries
    def get_F(self, i: int, stream=None) -> np.ndarray:
        m = self.query(i)["m"]
        out = np.zeros((m, m), dtype=np.float64, order="F")
        _check(self._lib.sc_get_F(self._h, i, out.ctypes.data, max(1, m), 0, _stream_handle(stream)))
        return out

    def get_F_device(self, i: int, out=None, ld: int = 0, stream=None):
        """F_i (m x m, FP64, original multiplier order) into a device tensor
        through sc_get_F(on_device = 1): column j at out[j * ld : j * ld + m]
        (ld >= m, default m).  Returns the (m, m) column-major view."""
        import torch
        m = self.query(i)["m"]
        ld = ld or max(1, m)
        if ld < m:
            raise ScasmError(SC_ERR_INVALID_ARG, f"ld {ld} < m {m}")
        if out is None:
            out = torch.zeros(ld * max(m, 1), dtype=torch.float64, device=f"cuda:{self.device_index}")
        check_dual_tensor(out, ld * m, self.device_index, "out")
        _check(self._lib.sc_get_F(self._h, i, ctypes.c_void_p(out.data_ptr()), ld, 1, _stream_handle(stream)))
        return out[: ld * m].view(m, ld).T[:m, :] if m else out[:0].view(0, 0)

    def query(self, i: int) -> dict:
        n, m, off, nnz = (ctypes.c_int64() for _ in range(4))
        fl = ctypes.c_double()
        _check(self._lib.sc_query(self._h, i, ctypes.byref(n), ctypes.byref(m), ctypes.byref(off),
                                  ctypes.byref(nnz), ctypes.byref(fl)))
        return {"n": n.value, "m": m.value, "dual_offset": off.value, "nnzL": nnz.value,
                "useful_flops": fl.value}

    def selection(self, i: int) -> dict:
        """The select_iters choice for subdomain i and its prediction."""
        imp = ctypes.c_int32()
        ta, te, ti, ns = (ctypes.c_double() for _ in range(4))
        _check(self._lib.sc_query_selection(self._h, i, ctypes.byref(imp), ctypes.byref(ta), ctypes.byref(te),
                                            ctypes.byref(ti), ctypes.byref(ns)))
        return {"implicit": bool(imp.value), "t_asm_ms": ta.value, "t_expl_ms": te.value, "t_impl_ms": ti.value,
                "n_star": ns.value}

    def stats(self) -> dict:
        ns = ctypes.c_int32()
        dt, db = ctypes.c_int64(), ctypes.c_int64()
        tu, su, td, sd, tr, sr = (ctypes.c_double() for _ in range(6))
        _check(self._lib.sc_plan_stats(self._h, ctypes.byref(ns), ctypes.byref(dt), ctypes.byref(tu),
                                       ctypes.byref(su), ctypes.byref(td), ctypes.byref(sd), ctypes.byref(tr),
                                       ctypes.byref(sr), ctypes.byref(db)))
        return {"nsub": ns.value, "dual_total": dt.value, "trsm_useful": tu.value, "syrk_useful": su.value,
                "trsm_dense": td.value, "syrk_dense": sd.value, "trsm_reach": tr.value, "syrk_reach": sr.value,
                "device_bytes": db.value}

    def set_timing(self, enable: bool = True):
        _check(self._lib.sc_set_timing(self._h, 1 if enable else 0))

    KERNELS = ("trsm", "syrk", "apply", "apply_implicit", "assemble_overlap")

    def kernel_times(self, reset: bool = True) -> dict:
        """Accumulated kernel milliseconds and launch counts (HIP events)."""
        ms = (ctypes.c_double * len(self.KERNELS))()
        cnt = (ctypes.c_int64 * len(self.KERNELS))()
        _check(self._lib.sc_kernel_times(self._h, ms, cnt, 1 if reset else 0))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def destroy(self):
        if self._h and self._h.value:
            self._lib.sc_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()
