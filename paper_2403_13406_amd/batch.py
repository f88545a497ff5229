"""Python binding of a batched ensemble (eslb_batch_* in include/eslb.h)."""
import ctypes

from . import _lib as L
from .solver import EslbError, make_problem


class Batch:
    """Independent problems of one kind advanced in lockstep, one stage kernel per pass over all of them."""

    def __init__(self, problems, stream=None):
        """problems: list of dicts of make_problem keyword arguments (same lattice/system/relax)."""
        import torch
        self.lib = L.load()
        self.n = len(problems)
        arr = (L.Problem * self.n)()
        for i, kw in enumerate(problems):
            arr[i] = make_problem(**kw)
        self.problems = arr
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        rc = self.lib.eslb_batch_create(arr, self.n, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc < 0:
            raise EslbError(rc, self.lib.eslb_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc < 0:
            raise EslbError(rc, self.lib.eslb_batch_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.eslb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, states):
        ptrs = (ctypes.c_void_p * self.n)()
        for i, t in enumerate(states):
            ptrs[i] = None if t is None else t.data_ptr()
        return ptrs

    def run(self, states, nsteps):
        steps = (ctypes.c_int64 * self.n)(*[int(v) for v in nsteps])
        return self._check(self.lib.eslb_batch_run(self.h, self._ptrs(states), steps))

    def offsets(self, i):
        q = 2 if self.problems[i].lattice == L.D1Q2 else 4
        arr = (ctypes.c_int64 * q)()
        self._check(self.lib.eslb_batch_get_offsets(self.h, i, arr))
        return list(arr)

    def sync(self):
        return self._check(self.lib.eslb_batch_sync_status(self.h))

    def set_config(self, block_x, block_y, blocks_per_cu, steps_per_graph):
        self._check(self.lib.eslb_batch_set_config(self.h, block_x, block_y, blocks_per_cu, steps_per_graph))

    def config(self):
        arr = (ctypes.c_int32 * 4)()
        self._check(self.lib.eslb_batch_get_config(self.h, arr))
        return list(arr)

    def autotune(self, states, replays=3):
        ms = ctypes.c_double()
        self._check(self.lib.eslb_batch_autotune(self.h, self._ptrs(states), int(replays), ctypes.byref(ms)))
        return self.config(), ms.value
