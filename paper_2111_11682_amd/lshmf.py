"""Python binding of liblshmf (ctypes): argument marshalling only.

Every step of the method runs in the HIP library; this module allocates the
caller-owned device tables with PyTorch, passes raw device pointers and the
current HIP stream, and turns non-zero statuses into exceptions.  There is no
CPU fallback: if the library is not built the import-time loader raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LSHMF_LIB") or os.path.join(HERE, "liblshmf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lshmf.h")

LSHMF_OK = 0
LSHMF_FP32, LSHMF_BF16, LSHMF_BF16_U = 0, 1, 2
STORAGE = {"fp32": LSHMF_FP32, "bf16": LSHMF_BF16, "bf16u": LSHMF_BF16_U}
SIMLSH, RPCOS, MINHASH = 0, 1, 2
NEIGHBOURHOOD, PLAIN_MF = 0, 1
REBUILD_NBRS = 1
STATUS = {0: "LSHMF_OK", -1: "LSHMF_EINVAL", -2: "LSHMF_ESTATE", -3: "LSHMF_ECAPACITY",
          -4: "LSHMF_EDEVICE"}


class LshmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Dims(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("F", C.c_int32), ("K", C.c_int32),
                ("G", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("rscale", C.c_int32),
                ("psi_exp", C.c_int32), ("n_strata", C.c_int32), ("storage", C.c_int32),
                ("hash_family", C.c_int32), ("model", C.c_int32), ("reserved", C.c_int32),
                ("nnz", C.c_int64), ("M_cap", C.c_int32),
                ("N_cap", C.c_int32), ("nnz_cap", C.c_int64), ("batch_cap", C.c_int64)]


class HParams(C.Structure):
    _fields_ = [("alpha", C.c_float * 6), ("lambda_", C.c_float * 6), ("beta", C.c_float),
                ("reserved", C.c_int32)]


class Tables(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("U", "V", "bu", "bv", "W", "C", "JK", "acc", "sig", "b0", "bh0", "mu",
                 "U16", "V16", "W16", "C16")]


class Layout(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("pk", "sj", "dep", "nib", "blk_ptr", "blk_seg", "seg_col", "seg_start",
                 "row_ptr", "csr_col", "csr_rc", "col_ptr", "csc_row", "csc_rc", "err")] + \
               [("nstride", C.c_int32), ("P", C.c_int32), ("M", C.c_int32), ("N", C.c_int32),
                ("nnz", C.c_int64)]


REQ_UPDATE, REQ_QUERY = 0, 1

# lshmf_request, as a numpy record type
REQUEST_DTYPE = np.dtype([("kind", "<i4"), ("M_new", "<i4"), ("N_new", "<i4"), ("reserved", "<i4"),
                          ("offset", "<i8"), ("n", "<i8"), ("arrival", "<f8")], align=True)


class ServeIO(C.Structure):
    _fields_ = [("req", C.c_void_p), ("n_req", C.c_int64),
                ("h_u", C.c_void_p), ("h_i", C.c_void_p), ("h_rc", C.c_void_p),
                ("h_qu", C.c_void_p), ("h_qi", C.c_void_p), ("h_pred", C.c_void_p),
                ("d_U0", C.c_void_p), ("d_V0", C.c_void_p), ("d_rand", C.c_void_p),
                ("seed_fill", C.c_uint64), ("hp", HParams), ("epoch", C.c_int32), ("passes", C.c_int32),
                ("max_query_batch", C.c_int64), ("d_stage", C.c_void_p), ("stage_bytes", C.c_size_t),
                ("h_start", C.c_void_p), ("h_done", C.c_void_p), ("h_status", C.c_void_p)]


_lock = threading.Lock()
_lib = None


def lib():
    """Loads liblshmf.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("liblshmf.so is not built (run __graft_entry__.build()); "
                                  "there is no CPU fallback")
            L = C.CDLL(LIB_PATH)
            vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
            L.lshmf_create.argtypes = [C.POINTER(Dims), C.POINTER(vp)]
            L.lshmf_destroy.argtypes = [vp]
            L.lshmf_destroy.restype = None
            L.lshmf_arena_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
            L.lshmf_bind.argtypes = [vp, C.POINTER(Tables), vp, C.c_size_t]
            L.lshmf_ingest.argtypes = [vp, vp, vp, vp, i64, vp]
            L.build_lsh_neighbours.argtypes = [vp, vp, u64, vp]
            L.sgd_epoch.argtypes = [vp, C.POINTER(HParams), i32, vp, vp]
            L.lshmf_loss.argtypes = [vp, C.POINTER(HParams), vp, vp]
            L.lshmf_check.argtypes = [vp, vp]
            L.lshmf_set_timing.argtypes = [vp, i32]
            L.lshmf_lsh_phase_ms.argtypes = [vp, C.POINTER(C.c_double)]
            L.online_update.argtypes = [vp, vp, vp, vp, i64, i32, i32, vp, u64, C.POINTER(HParams),
                                        i32, i32, C.c_uint32, vp]
            L.predict.argtypes = [vp, vp, vp, i64, vp, vp]
            L.lshmf_rmse.argtypes = [vp, vp, vp, i64, vp, vp]
            L.lshmf_rmse_noalloc.argtypes = [vp, vp, i64, i32, vp, vp]
            L.lshmf_export_layout.argtypes = [vp, C.POINTER(Layout)]
            L.lshmf_sync_storage.argtypes = [vp, vp]
            L.lshmf_serve_stage_bytes.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
            L.lshmf_serve.argtypes = [vp, C.POINTER(ServeIO), vp, vp]
            L.lshmf_last_error.restype = C.c_char_p
            L.lshmf_last_error.argtypes = []
            _lib = L
    return _lib


def _check(status: int):
    if status != LSHMF_OK:
        raise LshmfError(status, lib().lshmf_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def header_functions() -> Sequence[str]:
    """Names of the functions declared in include/lshmf.h."""
    import re
    src = open(HEADER).read()
    return re.findall(r"^\s*(?:int|void|const char\*)\s+([a-z_][a-z0-9_]*)\s*\(", src, re.M)


def rmse_noalloc(pred: torch.Tensor, rc: torch.Tensor, rscale: int, out: torch.Tensor):
    """lshmf_rmse_noalloc: the RMSE of predictions against rating codes into
    out[0] (FP64), with no context and no allocation by the library."""
    assert pred.dtype == torch.float32 and rc.dtype == torch.uint8 and out.dtype == torch.float64
    assert pred.numel() == rc.numel() and out.numel() >= 1
    _check(lib().lshmf_rmse_noalloc(_ptr(pred), _ptr(rc), pred.numel(), rscale, _ptr(out),
                                    _stream(out.device)))
    return out


class LshMF:
    """Device-resident LSH-MF model driven through the C ABI."""

    def __init__(self, M: int, N: int, F: int, K: int, G: int, p: int, q: int, rscale: int,
                 nnz: int, psi_exp: int = 2, n_strata: int = 256, device="cuda",
                 M_cap: int = 0, N_cap: int = 0, nnz_cap: int = 0, batch_cap: int = 0,
                 storage: str = "fp32", hash_family: int = SIMLSH, model: int = NEIGHBOURHOOD):
        """Tables are allocated for the capacities (0: the initial M, N, nnz);
        batch_cap > 0 enables online_update batches of up to that many ratings.
        storage "bf16" adds BF16 copies U16, V16, W16, C16 that predict reads;
        "bf16u" keeps the user rows only in BF16 (U16; U is not used).
        hash_family: SIMLSH, RPCOS or MINHASH (the neighbour search's hash);
        model: NEIGHBOURHOOD (Eq. rr) or PLAIN_MF (u . v only, K = 0)."""
        self.device = torch.device(device)
        assert storage in STORAGE
        self.storage = storage
        self.hash_family = hash_family
        self.dims = Dims(M, N, F, K, G, p, q, rscale, psi_exp, n_strata,
                         STORAGE[storage], hash_family, model, 0, nnz,
                         M_cap, N_cap, nnz_cap, batch_cap)
        M, N = max(M, M_cap), max(N, N_cap)
        self.B = G * p * q
        self.words = (self.B + 31) // 32
        h = C.c_void_p()
        _check(lib().lshmf_create(C.byref(self.dims), C.byref(h)))
        self._h = h
        nbytes = C.c_size_t()
        _check(lib().lshmf_arena_bytes(h, C.byref(nbytes)))
        dev = self.device
        f32 = dict(dtype=torch.float32, device=dev)
        self.U = torch.zeros(M, F, **f32)
        self.V = torch.zeros(N, F, **f32)
        self.bu = torch.zeros(M, **f32)
        self.bv = torch.zeros(N, **f32)
        self.W = torch.zeros(N, K, **f32)
        self.C = torch.zeros(N, K, **f32)
        self.JK = torch.zeros(N, K, dtype=torch.int32, device=dev)
        self.acc = torch.zeros(N, self.B, dtype=torch.int32, device=dev)
        self.sig = torch.zeros(N, self.words, dtype=torch.int32, device=dev)
        self.b0 = torch.zeros(M, **f32)
        self.bh0 = torch.zeros(N, **f32)
        self.mu = torch.zeros(1, dtype=torch.float64, device=dev)
        self.arena = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        off = (-self.arena.data_ptr()) % 256
        self._arena_ptr = self.arena.data_ptr() + off
        bf16 = dict(dtype=torch.bfloat16, device=dev)
        if storage != "fp32":
            self.U16 = torch.zeros(M, F, **bf16)
            self.V16 = torch.zeros(N, F, **bf16)
            self.W16 = torch.zeros(N, K, **bf16)
            self.C16 = torch.zeros(N, K, **bf16)
            half = [t.data_ptr() for t in (self.U16, self.V16, self.W16, self.C16)]
        else:
            self.U16 = self.V16 = self.W16 = self.C16 = None
            half = [0, 0, 0, 0]
        self.tables = Tables(*([t.data_ptr() for t in (self.U, self.V, self.bu, self.bv, self.W,
                                                        self.C, self.JK, self.acc, self.sig,
                                                        self.b0, self.bh0, self.mu)] + half))
        _check(lib().lshmf_bind(h, C.byref(self.tables), C.c_void_p(self._arena_ptr),
                                C.c_size_t(int(nbytes.value))))

    def close(self):
        if getattr(self, "_h", None):
            lib().lshmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tables
    def set_factors(self, U0: torch.Tensor, V0: torch.Tensor):
        """Initial U, V of the first rows (copied); b, bh, W, C start at zero."""
        self.U[: U0.shape[0]].copy_(U0)
        if self.storage == "bf16u":  # the user rows live in BF16 only (round to nearest even)
            self.U16[: U0.shape[0]].copy_(U0.to(torch.bfloat16))
        self.V[: V0.shape[0]].copy_(V0)
        for t in (self.bu, self.bv, self.W, self.C):
            t.zero_()

    # -- C ABI entry points
    def ingest(self, u: torch.Tensor, i: torch.Tensor, rc: torch.Tensor):
        assert u.dtype == torch.int32 and i.dtype == torch.int32 and rc.dtype == torch.uint8
        assert u.is_contiguous() and i.is_contiguous() and rc.is_contiguous()
        self._keep = (u, i, rc)
        _check(lib().lshmf_ingest(self._h, _ptr(u), _ptr(i), _ptr(rc), u.numel(),
                                  _stream(self.device)))

    def rand_cols(self) -> int:
        """Columns per user of the hash family's random draws."""
        return {SIMLSH: self.words, RPCOS: self.B, MINHASH: self.B // self.dims.G}[self.hash_family]

    def _check_rand(self, R: torch.Tensor, rows: int):
        want = torch.float32 if self.hash_family == RPCOS else torch.int32
        assert R.dtype == want and R.is_contiguous() and R.dim() == 2
        assert R.shape[1] == self.rand_cols() and R.shape[0] >= rows

    def build_lsh_neighbours(self, R: torch.Tensor, seed_fill: int):
        """R: the family's random draws per user -- simLSH bit strings H
        (int32 words), RP_cos Gaussians (float32, B per user), minHash random
        values (int32 bit patterns of uint32, B/G per user)."""
        self._check_rand(R, self.dims.M)
        _check(lib().build_lsh_neighbours(self._h, _ptr(R), C.c_uint64(seed_fill & (2**64 - 1)),
                                          _stream(self.device)))

    def sgd_epoch(self, alpha, lam, beta: float, epoch: int, loss_out: Optional[torch.Tensor] = None):
        """One epoch; loss_out (float64 [1] on the device) receives Eq. (loss_r)
        after it when given."""
        hp = HParams((C.c_float * 6)(*alpha), (C.c_float * 6)(*lam), beta, 0)
        _check(lib().sgd_epoch(self._h, C.byref(hp), epoch, _ptr(loss_out), _stream(self.device)))

    def loss(self, lam, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Eq. (loss_r) on the current tables (FP64, device)."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        hp = HParams((C.c_float * 6)(*([0.0] * 6)), (C.c_float * 6)(*lam), 0.0, 0)
        _check(lib().lshmf_loss(self._h, C.byref(hp), _ptr(out), _stream(self.device)))
        return out

    def set_timing(self, enable: bool = True):
        """Phase timing of build_lsh_neighbours (HIP events at its phase boundaries)."""
        _check(lib().lshmf_set_timing(self._h, int(bool(enable))))

    def lsh_phase_ms(self):
        """Milliseconds of the last timed neighbour search: hash state,
        signatures, band keys and buckets, top-K, neighbour codes."""
        out = (C.c_double * 5)()
        _check(lib().lshmf_lsh_phase_ms(self._h, out))
        return dict(zip(("hash_state", "signatures", "banding", "topk", "codes"), list(out)))

    def check(self):
        """Synchronises and raises LSHMF_EDEVICE if an SGD wait gave up."""
        _check(lib().lshmf_check(self._h, _stream(self.device)))

    def online_update(self, u: torch.Tensor, i: torch.Tensor, rc: torch.Tensor, M_new: int, N_new: int,
                      H: torch.Tensor, seed_fill: int, alpha, lam, beta: float, epoch: int,
                      passes: int = 1, U_new: Optional[torch.Tensor] = None,
                      V_new: Optional[torch.Tensor] = None, rebuild: bool = False):
        """Folds a batch of ratings into the model (Sec. 4.3); U_new / V_new
        are the initial factor rows of the new users / items; H the family's
        random draws (as for build_lsh_neighbours); rebuild searches every
        neighbour list again (LSHMF_REBUILD_NBRS)."""
        assert u.dtype == torch.int32 and i.dtype == torch.int32 and rc.dtype == torch.uint8
        assert u.is_contiguous() and i.is_contiguous() and rc.is_contiguous()
        self._check_rand(H, M_new)
        lay = self.layout()
        # rows beyond the capacity are left to the library to reject
        if lay.M < M_new <= self.U.shape[0]:
            assert U_new is not None and tuple(U_new.shape) == (M_new - lay.M, self.dims.F)
            self.U[lay.M: M_new].copy_(U_new)
            if self.storage == "bf16u":
                self.U16[lay.M: M_new].copy_(U_new.to(torch.bfloat16))
        if lay.N < N_new <= self.V.shape[0]:
            assert V_new is not None and tuple(V_new.shape) == (N_new - lay.N, self.dims.F)
            self.V[lay.N: N_new].copy_(V_new)
        hp = HParams((C.c_float * 6)(*alpha), (C.c_float * 6)(*lam), beta, 0)
        _check(lib().online_update(self._h, _ptr(u), _ptr(i), _ptr(rc), u.numel(), M_new, N_new,
                                   _ptr(H), C.c_uint64(seed_fill & (2**64 - 1)), C.byref(hp),
                                   epoch, passes, REBUILD_NBRS if rebuild else 0,
                                   _stream(self.device)))

    def sync_storage(self):
        """BF16 mode: rewrite the BF16 copies from the FP32 masters."""
        _check(lib().lshmf_sync_storage(self._h, _stream(self.device)))

    def serve(self, req: np.ndarray, upd, qry, U0: torch.Tensor, V0: torch.Tensor, H: torch.Tensor,
              seed_fill: int, alpha, lam, beta: float, epoch: int, passes: int = 1,
              max_query_batch: int = 65536):
        """Runs the serving loop over a request log (REQUEST_DTYPE records).

        upd = (u, i, rc) and qry = (qu, qi): host tensors (pinned for overlap)
        holding every request's payload at its offset; U0 / V0: device tables
        of initial rows for new ids.  Returns (answers, start, done, status)."""
        req = np.ascontiguousarray(req, REQUEST_DTYPE)
        n_req = req.size
        u, i, rc = upd
        qu, qi = qry
        pred = torch.zeros(max(qu.numel(), 1), dtype=torch.float32, pin_memory=True)
        start = np.zeros(n_req, np.float64)
        done = np.zeros(n_req, np.float64)
        status = np.zeros(n_req, np.int32)
        nbytes = C.c_size_t()
        _check(lib().lshmf_serve_stage_bytes(self._h, max_query_batch, C.byref(nbytes)))
        stage = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        sp = stage.data_ptr() + (-stage.data_ptr()) % 256
        hp = HParams((C.c_float * 6)(*alpha), (C.c_float * 6)(*lam), beta, 0)
        io = ServeIO(req.ctypes.data, n_req, u.data_ptr(), i.data_ptr(), rc.data_ptr(),
                     qu.data_ptr(), qi.data_ptr(), pred.data_ptr(), U0.data_ptr(), V0.data_ptr(),
                     H.data_ptr(), seed_fill & (2**64 - 1), hp, epoch, passes, max_query_batch, sp,
                     int(nbytes.value), start.ctypes.data, done.ctypes.data, status.ctypes.data)
        torch.cuda.synchronize(self.device)
        cs = torch.cuda.Stream(self.device)
        ps = torch.cuda.Stream(self.device)
        _check(lib().lshmf_serve(self._h, C.byref(io), C.c_void_p(cs.cuda_stream),
                                 C.c_void_p(ps.cuda_stream)))
        torch.cuda.synchronize(self.device)
        del stage
        return pred[: qu.numel()], start, done, status

    def predict(self, u: torch.Tensor, i: torch.Tensor, out: Optional[torch.Tensor] = None):
        assert u.dtype == torch.int32 and i.dtype == torch.int32
        if out is None:
            out = torch.empty(u.numel(), dtype=torch.float32, device=self.device)
        _check(lib().predict(self._h, _ptr(u), _ptr(i), u.numel(), _ptr(out), _stream(self.device)))
        return out

    def rmse(self, pred: torch.Tensor, rc: torch.Tensor, out: Optional[torch.Tensor] = None):
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(lib().lshmf_rmse(self._h, _ptr(pred), _ptr(rc), pred.numel(), _ptr(out),
                                _stream(self.device)))
        return out

    def layout(self) -> Layout:
        lay = Layout()
        _check(lib().lshmf_export_layout(self._h, C.byref(lay)))
        return lay

    def device_status(self) -> int:
        """The library's device status word (0 while healthy); synchronises."""
        lay = self.layout()
        torch.cuda.synchronize(self.device)
        return int(self.arena_view(lay.err, 1, torch.int32).item())

    def arena_view(self, ptr: int, n: int, dtype: torch.dtype) -> torch.Tensor:
        """A tensor view of n elements of the library's arena starting at ptr."""
        off = ptr - self.arena.data_ptr()
        esz = torch.empty(0, dtype=dtype).element_size()
        assert off >= 0 and off % esz == 0 and off + n * esz <= self.arena.numel()
        return self.arena[off: off + n * esz].view(dtype)
