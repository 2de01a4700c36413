"""Row-parallel evaluation of an oracle sampler (test infrastructure only).

The black-box sampler of Sec. 2.1 solves one PDE per sampling node; the
solves are independent, so the rows of a node matrix can be split over
worker processes without changing any result: every row is solved by the
same code, alone, in float64, and the rows are put back in their order.
This only shortens the wall time of oracle runs at the larger workloads
(the fixture scripts under tests/golden/ and the all-core CPU baseline).
"""
import multiprocessing as mp
import os

import numpy as np

_WORKER_SAMPLER = None


def _init(sampler):
    global _WORKER_SAMPLER
    _WORKER_SAMPLER = sampler
    # one BLAS thread per worker process: the workers already fill the cores
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except ImportError:
        pass


def _run(Y):
    return _WORKER_SAMPLER(Y)


class PooledSampler:
    """Callable Y (n x d) -> U (n x G) that evaluates `sampler` on row chunks
    in `workers` forked processes.  Use as a context manager."""

    def __init__(self, sampler, workers=None, chunk=64):
        self.sampler = sampler
        self.G = sampler.G
        self.workers = int(workers or os.cpu_count() or 1)
        self.chunk = int(chunk)
        self._pool = None

    def __enter__(self):
        if self.workers > 1:
            ctx = mp.get_context("fork")
            self._pool = ctx.Pool(self.workers, initializer=_init, initargs=(self.sampler,))
        return self

    def __exit__(self, *exc):
        if self._pool is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None

    def __call__(self, Y):
        Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
        if self._pool is None or len(Y) <= self.chunk:
            return self.sampler(Y)
        parts = [Y[a:a + self.chunk] for a in range(0, len(Y), self.chunk)]
        return np.concatenate(self._pool.map(_run, parts), axis=0)
