"""Oracle output rows of a large workload, computed in parallel (test infrastructure).

Each row (k, i) of V_x u is a sum over every source orbital, which the FP64 oracle
evaluates row by row. Here one spawned process per row runs oracle.fock_apply,
unmodified, on a shared-memory copy of the orbitals."""

from __future__ import annotations

import multiprocessing as mp
import os
from multiprocessing import shared_memory

import numpy as np

_S = {}


def _init(name, shape, kp, cell, omega):
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    import oracle  # noqa: F401
    shm = shared_memory.SharedMemory(name=name)
    _S.update(shm=shm, u=np.ndarray(shape, dtype=np.complex128, buffer=shm.buf), kp=kp, cell=cell, omega=omega)


def _row(row):
    import oracle
    s = _S
    return row, oracle.fock_apply(s["u"], s["u"], s["kp"], s["cell"], s["omega"], rows=[row])[row]


def oracle_rows(u, kp, cell, omega, rows, workers=None):
    """{(k, i): (V_x u)[k, i]} from the FP64 oracle, one process per row."""
    u = np.ascontiguousarray(u)
    workers = workers or min(len(rows), 16, os.cpu_count() or 1)
    shm = shared_memory.SharedMemory(create=True, size=u.nbytes)
    try:
        np.ndarray(u.shape, dtype=u.dtype, buffer=shm.buf)[...] = u
        with mp.get_context("spawn").Pool(workers, initializer=_init,
                                         initargs=(shm.name, u.shape, np.asarray(kp), np.asarray(cell), omega)) as pool:
            return dict(pool.map(_row, list(rows), chunksize=1))
    finally:
        shm.close()
        shm.unlink()
