import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NATIVE = os.path.join(ROOT, "tests", "native")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on cuda:0)")
    config.addinivalue_line("markers", "slow: long CPU test")


def _build_native(name, cmd):
    out = os.path.join(NATIVE, name)
    if not os.path.exists(out):
        subprocess.check_call(cmd, cwd=NATIVE)
    return out


@pytest.fixture(scope="session")
def bruteforce():
    path = _build_native("libbruteforce.so",
                         ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "bruteforce.c",
                          "-o", "libbruteforce.so"])
    lib = ctypes.CDLL(path)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    lib.bf_enumerate.restype = ctypes.c_int
    lib.bf_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), u64p]

    def run(n_spins, bonds):
        """bonds: list of (i, j, J).  Returns (E_min, dos dict E -> count)."""
        bi = np.array([b[0] for b in bonds], np.int32)
        bj = np.array([b[1] for b in bonds], np.int32)
        bJ = np.array([b[2] for b in bonds], np.int32)
        bound = int(np.abs(bJ).sum())
        nb = 2 * bound + 1
        dos = np.zeros(nb, np.uint64)
        emin = ctypes.c_int64(0)
        rc = lib.bf_enumerate(n_spins, len(bonds), bi, bj, bJ, -bound, nb, ctypes.byref(emin), dos)
        assert rc == 0
        return int(emin.value), {e - bound: int(c) for e, c in enumerate(dos) if c}
    return run


@pytest.fixture(scope="session")
def rocrand_philox():
    path = _build_native("librocrand_probe.so",
                         ["hipcc", "-O2", "-fPIC", "-shared", "rocrand_probe.cpp",
                          "-o", "librocrand_probe.so"])
    lib = ctypes.CDLL(path)
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    lib.rocrand_philox_blocks.restype = None
    lib.rocrand_philox_blocks.argtypes = [u32p, ctypes.c_uint32, ctypes.c_uint32, u32p,
                                          ctypes.c_int64]
    lib.rocrand_philox_public.restype = None
    lib.rocrand_philox_public.argtypes = [ctypes.c_uint64, u32p, u32p, ctypes.c_int64]
    return lib


def bonds_from_J(J, dims):
    """Bond list (i, j, J_ij) of the +x, +y, +z couplings with nonzero J,
    using this file's own neighbour arithmetic (x fastest)."""
    Lx, Ly, Lz = dims
    N = Lx * Ly * Lz
    J = np.asarray(J).reshape(6, N)
    out = []
    for i in range(N):
        x, y, z = i % Lx, (i // Lx) % Ly, i // (Lx * Ly)
        for d, (dx, dy, dz) in ((0, (1, 0, 0)), (2, (0, 1, 0)), (4, (0, 0, 1))):
            j = (x + dx) % Lx + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))
            if J[d, i] != 0:
                out.append((i, j, int(J[d, i])))
    return out


def neighbours(dims):
    """nbr[d, i] with d = +x,-x,+y,-y,+z,-z (x fastest), independent of the oracle."""
    Lx, Ly, Lz = dims
    i = np.arange(Lx * Ly * Lz)
    x, y, z = i % Lx, (i // Lx) % Ly, i // (Lx * Ly)
    idx = lambda a, b, c: (a % Lx) + Lx * ((b % Ly) + Ly * (c % Lz))
    return np.stack([idx(x + 1, y, z), idx(x - 1, y, z), idx(x, y + 1, z), idx(x, y - 1, z),
                     idx(x, y, z + 1), idx(x, y, z - 1)])
