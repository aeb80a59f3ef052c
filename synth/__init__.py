"""Seeded synthetic long-read workloads (shared input generator).

The paper measures its alignment stage on PacBio E. coli reads (section 5:
30x, 16,890 reads of mean 9,958 bp; 100x, 91,394 reads of mean 6,934 bp).
Those datasets are not available, so every input here is synthetic and
seeded: a uniform-ACGT genome (optionally with exact repeat copies), reads
sampled from it with iid substitution/insertion/deletion errors, and
alignment tasks whose seed is a k-base template window copied without error
into both reads (the paper seeds each alignment with a shared retained k-mer,
section 4 stages 3-4).

This module draws random numbers and records simulation truth only; it holds
no alignment arithmetic.  Both the oracle tests and the HIP path take their
inputs from here.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "gen.cpp")


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("genome_len", ctypes.c_uint64),
        ("n_rep_src", ctypes.c_uint32),
        ("rep_len", ctypes.c_uint32),
        ("n_rep_copies", ctypes.c_uint32),
        ("mode", ctypes.c_int32),
        ("depth", ctypes.c_double),
        ("len_dist", ctypes.c_int32),
        ("len_mean", ctypes.c_double),
        ("len_sd", ctypes.c_double),
        ("len_min", ctypes.c_uint32),
        ("len_max", ctypes.c_uint32),
        ("p_sub", ctypes.c_double),
        ("p_ins", ctypes.c_double),
        ("p_del", ctypes.c_double),
        ("k", ctypes.c_uint32),
        ("min_overlap", ctypes.c_uint32),
        ("n_tasks", ctypes.c_uint64),
        ("seeds_per_pair", ctypes.c_int32),
        ("n_x", ctypes.c_int32),
        ("x_choices", ctypes.c_int32 * 8),
        ("spurious_frac", ctypes.c_double),
    ]


def build_lib(force: bool = False) -> str:
    """Compile the generator into a shared library next to its source."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_make.restype = ctypes.c_void_p
        lib.synth_make.argtypes = [ctypes.POINTER(_Params)]
        lib.synth_sizes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
        lib.synth_copy.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 11
        lib.synth_genome.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclasses.dataclass
class Workload:
    """A read set plus alignment tasks.

    codes:   uint8[n_bases], base codes A=0 C=1 G=2 T=3, reads concatenated
    off:     uint64[n_reads], first base of each read in `codes`
    length:  uint32[n_reads]
    tspan:   uint32[n_reads, 2], template interval each read was sampled from
    ra, rb:  uint32[n_tasks], read ids of each task
    pa, pb:  uint32[n_tasks], 0-based start of the shared k-mer in ra / rb
    x:       int32[n_tasks], X-drop threshold per task
    ovl:     uint32[n_tasks], true template overlap (0 for repeat-induced)
    spurious: uint8[n_tasks], 1 if the seed comes from two repeat copies
    """
    name: str
    params: dict
    codes: np.ndarray
    off: np.ndarray
    length: np.ndarray
    tspan: np.ndarray
    ra: np.ndarray
    rb: np.ndarray
    pa: np.ndarray
    pb: np.ndarray
    x: np.ndarray
    ovl: np.ndarray
    spurious: np.ndarray
    k: int
    n_candidate_pairs: int
    n_candidate_tasks: int
    genome: np.ndarray | None = None

    @property
    def n_reads(self) -> int:
        return int(self.length.shape[0])

    @property
    def n_tasks(self) -> int:
        return int(self.ra.shape[0])

    def read(self, r: int) -> np.ndarray:
        o = int(self.off[r])
        return self.codes[o:o + int(self.length[r])]

    def subset(self, idx) -> "Workload":
        """Same read set, tasks restricted to `idx`."""
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, name=self.name + "[sub]", ra=self.ra[idx], rb=self.rb[idx],
            pa=self.pa[idx], pb=self.pb[idx], x=self.x[idx], ovl=self.ovl[idx],
            spurious=self.spurious[idx])


DEFAULTS = dict(
    seed=1, genome_len=200_000, n_rep_src=0, rep_len=0, n_rep_copies=0,
    mode=1, depth=30.0, len_dist=1, len_mean=10_000.0, len_sd=5_000.0,
    len_min=1_000, len_max=50_000, p_sub=0.05, p_ins=0.05, p_del=0.05,
    k=17, min_overlap=1_000, n_tasks=0, seeds_per_pair=0, x=(25,),
    spurious_frac=0.0,
)


def make(name: str = "custom", keep_genome: bool = False, **kw) -> Workload:
    """Generate a workload from generator parameters (see DEFAULTS)."""
    p = dict(DEFAULTS)
    unknown = set(kw) - set(p)
    if unknown:
        raise ValueError("unknown generator parameters: %s" % sorted(unknown))
    p.update(kw)
    xs = tuple(int(v) for v in p["x"])
    if not 1 <= len(xs) <= 8:
        raise ValueError("1..8 X choices")
    cp = _Params()
    for f, _ in _Params._fields_:
        if f in ("n_x", "x_choices"):
            continue
        setattr(cp, f, p[f])
    cp.n_x = len(xs)
    for i, v in enumerate(xs):
        cp.x_choices[i] = v
    lib = _load()
    h = lib.synth_make(ctypes.byref(cp))
    try:
        sz = (ctypes.c_uint64 * 6)()
        lib.synth_sizes(h, sz)
        nb, nr, nt = int(sz[0]), int(sz[1]), int(sz[2])
        codes = np.empty(nb, np.uint8)
        off = np.empty(nr, np.uint64)
        length = np.empty(nr, np.uint32)
        tspan = np.empty((nr, 2), np.uint32)
        ra, rb, pa, pb, ovl = (np.empty(nt, np.uint32) for _ in range(5))
        x = np.empty(nt, np.int32)
        spur = np.empty(nt, np.uint8)

        def ptr(a):
            return a.ctypes.data_as(ctypes.c_void_p)
        lib.synth_copy(h, ptr(codes), ptr(off), ptr(length), ptr(tspan), ptr(ra), ptr(rb),
                       ptr(pa), ptr(pb), ptr(x), ptr(ovl), ptr(spur))
        genome = None
        if keep_genome:
            genome = np.empty(int(sz[5]), np.uint8)
            lib.synth_genome(h, ptr(genome))
        return Workload(name=name, params=p, codes=codes, off=off, length=length, tspan=tspan,
                        ra=ra, rb=rb, pa=pa, pb=pb, x=x, ovl=ovl, spurious=spur, k=int(p["k"]),
                        n_candidate_pairs=int(sz[3]), n_candidate_tasks=int(sz[4]),
                        genome=genome)
    finally:
        lib.synth_free(h)


from .configs import CONFIGS, config  # noqa: E402  (re-export)
