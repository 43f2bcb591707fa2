"""Batched matvec over many compressed matrices in one persistent launch
(binding of ccm_batch_* in include/ccm.h)."""
from __future__ import annotations

import ctypes
import os

import torch

from ._lib import E_UNSUPPORTED, I32, I64, CcmError, Desc, check, lib


def _row_major(m, what: str) -> None:
    if getattr(m, "order", "C") != "C":
        raise CcmError(E_UNSUPPORTED, f"{what}: column-major matrix")

# Widest matrix (columns) a batched launch accepts: its x is staged whole in LDS.
BATCH_MAX_COLS = 8192

# Tuning table written by the autotuner for gfx950 (built-in defaults if absent).
DEFAULT_TUNE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", "gfx950.json")


class Batch:
    """A fixed set of compressed matrices whose matvecs run in one launch."""

    def __init__(self, mats, xdtype=torch.int32, tune_json: str | None = "default"):
        if tune_json == "default":
            tune_json = DEFAULT_TUNE if os.path.exists(DEFAULT_TUNE) else None
        self.mats = list(mats)
        n = len(self.mats)
        arr = (Desc * n)()
        for t, m in enumerate(self.mats):
            _row_major(m, "Batch")
            arr[t] = m.desc
        self._descs = arr
        self.xcode = I32 if xdtype == torch.int32 else I64
        h = ctypes.c_void_p()
        check(lib.ccm_batch_create(arr, n, self.xcode,
                                   tune_json.encode() if tune_json else None, ctypes.byref(h)),
              "ccm_batch_create")
        self._h = h

    def set_io(self, xs, ys, stream=None):
        n = len(self.mats)
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        yp = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib.ccm_batch_set_io(self._h, xp, yp, ctypes.c_void_p(s.cuda_stream)),
              "ccm_batch_set_io")
        self._io = (xs, ys)  # keep the tensors alive while bound

    def run(self, use_graph: bool = True, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib.ccm_batch_matvec(self._h, 1 if use_graph else 0, ctypes.c_void_p(s.cuda_stream)),
              "ccm_batch_matvec")

    def info(self):
        items, nbytes, mb = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int32()
        check(lib.ccm_batch_info(self._h, ctypes.byref(items), ctypes.byref(nbytes),
                                 ctypes.byref(mb)), "ccm_batch_info")
        return {"items": int(items.value), "packed_bytes": int(nbytes.value),
                "max_bits": int(mb.value)}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(lib.ccm_batch_destroy(self._h), "ccm_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DynBatch:
    """Workspace for batched matvecs over a different set of matrices on every
    launch (ccm_batch_ws_* / ccm_batch_matvec_dyn)."""

    def __init__(self, max_mats: int = 4096, max_items: int = 1 << 16, slots: int = 4,
                 tune_json: str | None = "default"):
        if tune_json == "default":
            tune_json = DEFAULT_TUNE if os.path.exists(DEFAULT_TUNE) else None
        h = ctypes.c_void_p()
        check(lib.ccm_batch_ws_create(max_mats, max_items, slots,
                                      tune_json.encode() if tune_json else None, ctypes.byref(h)),
              "ccm_batch_ws_create")
        self._h = h

    def matvec(self, mats, xs, ys, stream=None):
        n = len(mats)
        arr = (Desc * n)()
        for t, m in enumerate(mats):
            _row_major(m, "DynBatch")
            arr[t] = m.desc
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        yp = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib.ccm_batch_matvec_dyn(self._h, arr, xp, yp, n, ctypes.c_void_p(s.cuda_stream)),
              "ccm_batch_matvec_dyn")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(lib.ccm_batch_ws_destroy(self._h), "ccm_batch_ws_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
