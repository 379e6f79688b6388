"""Seeded synthetic genotype inputs shared by the tests, the oracle checks and the bench.

Input generation only: this package draws genotype matrices shaped like the
workloads the GKL hot path is measured on and packs them in the 2-bit storage
format.  It holds none of the method's arithmetic.  The per-genotype bulk runs
in ``gen.c`` (counter-based, thread-count independent); the per-SNP and
per-individual parameters (allele frequencies, subpopulation drift, admixture
weights, planted spikes) are drawn here with NumPy's PCG64.

Storage format: SNP-major, column j in bytes [j*ld, (j+1)*ld), individual i in
byte j*ld + i//4 at bits 2*(i%4); codes 0/1/2 = allele count, 3 = missing.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib = None


def build_library(force: bool = False) -> str:
    """Compile gen.c into libsynth.so with gcc/OpenMP (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               os.path.join(_HERE, "gen.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build_library()
            lib = ctypes.CDLL(_LIB_PATH)
            i64, u64, i32, vp, dbl = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_double)
            lib.synth_genotypes.argtypes = [i64, i64, i64, u64, vp, i64, vp, vp, vp, dbl, i32, vp]
            lib.synth_genotypes.restype = ctypes.c_int
            lib.synth_genotypes_range.argtypes = [i64, i64, i64, i64, i64, u64, vp, i64, vp, vp, vp,
                                                  dbl, i32, vp]
            lib.synth_genotypes_range.restype = ctypes.c_int
            lib.synth_pack.argtypes = [i64, i64, i64, vp, i32, vp]
            lib.synth_pack.restype = ctypes.c_int
            lib.synth_algorithm1.argtypes = [i64, i64, i64, vp, dbl, vp, u64, vp, i64, vp]
            lib.synth_algorithm1.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclasses.dataclass
class Genotypes:
    """A packed genotype matrix plus the recipe that made it."""
    packed: np.ndarray          # uint8, shape (p, ld)
    n: int
    p: int
    ld: int
    meta: dict

    @property
    def nbytes(self) -> int:
        return int(self.packed.nbytes)


def default_ld(n: int) -> int:
    return (n + 3) // 4


def pack_codes(codes: np.ndarray, ld: int | None = None, pad_mode: int = 0) -> np.ndarray:
    """Pack an (n, p) array of codes 0..3 into the (p, ld) storage format."""
    codes = np.asarray(codes)
    n, p = codes.shape
    ld = default_ld(n) if ld is None else int(ld)
    colmajor = np.ascontiguousarray(codes.T.astype(np.int8))
    out = np.empty((p, ld), dtype=np.uint8)
    rc = _load().synth_pack(n, p, ld, _ptr(colmajor), pad_mode, _ptr(out))
    if rc != 0:
        raise ValueError("synth_pack rejected its arguments")
    return out


PROGRESS_COLUMNS = 50000     # SNP columns per reported range


def generate(n: int, p: int, seed: int, base: np.ndarray, A: np.ndarray | None = None,
             B: np.ndarray | None = None, hap0_src: np.ndarray | None = None,
             miss_rate: float = 0.0, ld: int | None = None, pad_mode: int = 0,
             progress=None) -> np.ndarray:
    """Bulk draw of a packed (p, ld) genotype matrix; see gen.c for the model.  With a
    `progress` callable the columns are drawn in ranges and each range is reported."""
    ld = default_ld(n) if ld is None else int(ld)
    base = np.ascontiguousarray(base, dtype=np.float64)
    assert base.shape == (p,)
    L = 0
    if A is not None:
        A = np.ascontiguousarray(A, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        L = A.shape[1]
        assert A.shape == (n, L) and B.shape == (L, p)
    if hap0_src is not None:
        hap0_src = np.ascontiguousarray(hap0_src, dtype=np.int32)
        assert hap0_src.shape == (n,)
    out = np.empty((p, ld), dtype=np.uint8)
    chunk = p if progress is None else max(1, min(p, PROGRESS_COLUMNS))
    for j0 in range(0, p, chunk):
        j1 = min(p, j0 + chunk)
        rc = _load().synth_genotypes_range(n, p, j0, j1, ld, seed & 0xFFFFFFFFFFFFFFFF, _ptr(base),
                                           L, _ptr(A), _ptr(B), _ptr(hap0_src), float(miss_rate),
                                           pad_mode, _ptr(out[j0:j1]))
        if rc != 0:
            raise ValueError("synth_genotypes_range rejected its arguments")
        if progress is not None:
            progress(f"[synth] {j1:,} of {p:,} SNP columns drawn")
    return out


# ---------------------------------------------------------------------------
# Per-SNP / per-individual parameter draws
# ---------------------------------------------------------------------------

def balding_nichols(rng: np.random.Generator, f: np.ndarray, F: float) -> np.ndarray:
    """Subpopulation allele frequencies drifted from ancestral f with fixation index F."""
    a = f * (1.0 - F) / F
    b = (1.0 - f) * (1.0 - F) / F
    return rng.beta(a, b)


def _subpop_model(rng, n, p, sizes, Fs, f):
    K = len(sizes)
    Fk = np.stack([balding_nichols(rng, f, Fs[k]) for k in range(K)])   # K x p
    pop = np.repeat(np.arange(K), sizes)
    A = np.zeros((n, K))
    A[np.arange(n), pop] = 1.0
    return Fk, pop, A


def mp_edge(n: int, p: int, miss_rate: float = 0.0) -> float:
    """Largest singular value of an n x p unit-variance noise matrix (bulk edge)."""
    return float(np.sqrt(1.0 - miss_rate) * (np.sqrt(n) + np.sqrt(p)))


def bbp_theta(ratio: float, c: float) -> float:
    """Spike strength theta whose outlier sits at ratio * (1 + sqrt c) (BBP inverse, c = n/p)."""
    s = (ratio * (1.0 + np.sqrt(c))) ** 2
    t = s - 1.0 - c
    return float(np.sqrt((t + np.sqrt(t * t - 4.0 * c)) / 2.0))


def related_pairs(rng, pop, frac):
    """hap0_src array: frac of individuals form pairs within a subpopulation; the
    second of each pair copies haplotype 0 from the first."""
    n = pop.shape[0]
    src = np.arange(n, dtype=np.int32)
    npairs = int(round(frac * n / 2))
    done = 0
    for k in np.unique(pop):
        idx = np.flatnonzero(pop == k)
        want = int(round(npairs * idx.size / n))
        pick = rng.choice(idx, size=2 * want, replace=False)
        for a, b in zip(pick[0::2], pick[1::2]):
            src[b] = a
        done += want
    return src


def chromosome_sizes() -> list[int]:
    """22 per-chromosome SNP counts decreasing geometrically from 80,000 to 8,000."""
    return [int(round(8000 * 10 ** ((22 - c) / 21.0))) for c in range(1, 23)]


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")
FULL_SIZES = {"c1": (1000, 5000), "c2": (10000, 100000), "c3": (50000, 500000),
              "c4": (20000, None), "c5": (100000, 1000000)}


def config(name: str, seed: int | None = None, n: int | None = None, p: int | None = None,
           chrom: int | None = None, ld: int | None = None, pad_mode: int = 0,
           progress=None) -> Genotypes:
    """Generate one workload.

    c1: 2 subpopulations (Balding-Nichols F = 0.01), f ~ U(0.05, 0.5), 1% missing.
    c2: 5 subpopulations (F 0.005..0.02), MAF ~ U(0.01, 0.5), 2% of individuals in
        related pairs (one shared haplotype), 1% missing.
    c3: 10 subpopulations (F 0.005..0.02), 20% admixed with Dirichlet(0.5) weights,
        MAF ~ U(0.01, 0.5), 1% missing.
    c4: one chromosome block (chrom = 1..22) of the 22-block genome; 4 subpopulations
        (F = 0.01) shared across blocks, f ~ U(0.05, 0.5), 1% missing.
    c5: no subpopulations, MAF ~ Beta(0.5, 0.5) folded and clipped to [0.01, 0.5],
        3% missing, 10 planted rank-one spikes at 1.5x..20x the noise edge.
    n, p override the full sizes (same recipe at a smaller shape).
    """
    name = name.lower()
    idx = CONFIG_NAMES.index(name)
    seed = idx + 1 if seed is None else int(seed)
    n0, p0 = FULL_SIZES[name]
    n = n0 if n is None else int(n)
    if name == "c4":
        chrom = 1 if chrom is None else int(chrom)
        p0 = chromosome_sizes()[chrom - 1]
    p = p0 if p is None else int(p)
    meta = {"config": name, "seed": seed, "n": n, "p": p}
    rng = np.random.default_rng([seed, 0x6B6C])
    hap0 = None
    if name == "c1":
        f = rng.uniform(0.05, 0.5, size=p)
        sizes = [n // 2, n - n // 2]
        Fk, pop, A = _subpop_model(rng, n, p, sizes, [0.01, 0.01], f)
        base, B, miss = np.zeros(p), Fk, 0.01
    elif name == "c2":
        f = rng.uniform(0.01, 0.5, size=p)
        K = 5
        sizes = [n // K + (1 if k < n % K else 0) for k in range(K)]
        Fk, pop, A = _subpop_model(rng, n, p, sizes, list(np.linspace(0.005, 0.02, K)), f)
        hap0 = related_pairs(rng, pop, 0.02)
        base, B, miss = np.zeros(p), Fk, 0.01
        meta["related_individuals"] = int(np.sum(hap0 != np.arange(n)))
    elif name == "c3":
        f = rng.uniform(0.01, 0.5, size=p)
        K = 10
        n_adm = int(round(0.2 * n))
        n_pure = n - n_adm
        sizes = [n_pure // K + (1 if k < n_pure % K else 0) for k in range(K)]
        Fk = np.stack([balding_nichols(rng, f, Fs) for Fs in np.linspace(0.005, 0.02, K)])
        pop = np.repeat(np.arange(K), sizes)
        A = np.zeros((n, K))
        A[np.arange(n_pure), pop] = 1.0
        A[n_pure:] = rng.dirichlet(0.5 * np.ones(K), size=n_adm)
        base, B, miss = np.zeros(p), Fk, 0.01
        meta["admixed"] = n_adm
    elif name == "c4":
        # Population structure is shared across chromosomes: the subpopulation
        # assignment uses a chromosome-independent stream.
        prng = np.random.default_rng([seed, 0x706F70])
        K = 4
        sizes = [n // K + (1 if k < n % K else 0) for k in range(K)]
        pop = np.repeat(np.arange(K), sizes)
        prng.shuffle(pop)
        crng = np.random.default_rng([seed, 0x6368, chrom])
        f = crng.uniform(0.05, 0.5, size=p)
        Fk = np.stack([balding_nichols(crng, f, 0.01) for _ in range(K)])
        A = np.zeros((n, K))
        A[np.arange(n), pop] = 1.0
        base, B, miss = np.zeros(p), Fk, 0.01
        seed = seed * 1000 + chrom
        meta["chrom"] = chrom
    else:  # c5
        miss = 0.03
        f = rng.beta(0.5, 0.5, size=p)
        f = np.clip(np.minimum(f, 1.0 - f), 0.01, 0.5)
        c = n / p
        ratios = np.geomspace(1.5, 20.0, 10)
        theta = np.array([bbp_theta(r, c) for r in ratios])
        t = theta * np.sqrt(p / (1.0 - miss))
        x = rng.choice([-1.0, 1.0], size=(10, n)) / np.sqrt(n)
        y = rng.choice([-1.0, 1.0], size=(10, p)) / np.sqrt(p)
        d = np.sqrt(2.0 * f * (1.0 - f))
        A = (x * t[:, None]).T                     # n x 10
        B = y * (d / 2.0)[None, :]                 # 10 x p
        base = f
        meta.update(spike_ratios=ratios.tolist(), theta=theta.tolist(),
                    edge=mp_edge(n, p, miss))
    meta["miss_rate"] = miss
    packed = generate(n, p, seed, base, A, B, hap0, miss, ld=ld, pad_mode=pad_mode,
                      progress=progress)
    return Genotypes(packed, n, p, packed.shape[1], meta)


def start_vector(p: int, seed: int) -> np.ndarray:
    """Seeded Gaussian start direction for the right Krylov basis (not normalised)."""
    return np.random.default_rng([seed, 0x7631]).standard_normal(p)


def spare_directions(p: int, count: int, seed: int) -> np.ndarray:
    """Seeded Gaussian directions used when the recurrence breaks down (count x p)."""
    return np.random.default_rng([seed, 0x62726B]).standard_normal((count, p))


def _algorithm1_params(rows, cols, r, nsignal, rkins, seed):
    """Rectangles, per-entry hit probability and row sources of the model."""
    rng = np.random.default_rng([seed, 0xA161])
    rb = np.sort(rng.integers(0, rows, size=(r, 2)), axis=1)
    cb = np.sort(rng.integers(0, cols, size=(r, 2)), axis=1)
    val = rng.integers(0, 3, size=r)
    rect = np.ascontiguousarray(np.column_stack([rb, cb, val]).astype(np.int64))
    q_hit = float(-np.expm1(nsignal * np.log1p(-1.0 / (float(rows) * float(cols)))))
    nk = int(round(rkins * rows))
    dst = rng.integers(0, rows, size=nk)
    src_rows = rng.integers(0, rows, size=nk)
    src = np.arange(rows, dtype=np.int32)
    keep = dst.size - 1 - np.unique(dst[::-1], return_index=True)[1]   # last pair per row
    src[dst[keep]] = src_rows[keep]
    return rect, q_hit, src


def algorithm1_codes(rows: int, cols: int, r: int, nsignal: int, rkins: float,
                     seed: int) -> np.ndarray:
    """The paper's crude random genotype model (Section 2, "A simple model for
    genomics data"), built from its three-step description.

    Admixture: r rectangles, each spanning a random contiguous range of rows and
    of columns (rectangles may overlap; later ones cover earlier ones), hold one
    random value in {0, 1, 2} each.  Signal: nsignal uniformly random positions
    (drawn with replacement) get random values in {0, 1, 2}, the last draw at a
    position holding -- drawn entry by entry: an entry is hit with probability
    1 - (1 - 1/(rows cols))^nsignal and then takes a uniform value.  Kinship:
    round(rkins * rows) rows are replaced by copies of randomly chosen rows, the
    copies taken from the matrix after the signal step, all at once.  Rows are
    individuals here, so the copies model related individuals.  Returns the
    (rows, cols) int8 code matrix.
    """
    rect, q_hit, src = _algorithm1_params(rows, cols, r, nsignal, rkins, seed)
    out = np.empty((cols, rows), dtype=np.int8)
    rc = _load().synth_algorithm1(rows, cols, r, _ptr(rect), q_hit, _ptr(src),
                                  seed & 0xFFFFFFFFFFFFFFFF, _ptr(out), 0, None)
    if rc != 0:
        raise ValueError("synth_algorithm1 rejected its arguments")
    return out.T


def algorithm1(rows: int = 41505, cols: int = 81700, r: int = 10, nsignal: int | None = None,
               rkins: float = 0.017, seed: int = 6) -> Genotypes:
    """The same model packed in the 2-bit storage format (no missing values); the
    defaults are the paper's Fig. 1 matrix (41,505 x 81,700, r = 10,
    nsignal = rows cols, rkins = 0.017), rows read as individuals."""
    nsignal = rows * cols if nsignal is None else int(nsignal)
    rect, q_hit, src = _algorithm1_params(rows, cols, r, nsignal, rkins, seed)
    ld = default_ld(rows)
    out = np.empty((cols, ld), dtype=np.uint8)
    rc = _load().synth_algorithm1(rows, cols, r, _ptr(rect), q_hit, _ptr(src),
                                  seed & 0xFFFFFFFFFFFFFFFF, None, ld, _ptr(out))
    if rc != 0:
        raise ValueError("synth_algorithm1 rejected its arguments")
    meta = {"config": "alg1", "seed": seed, "n": rows, "p": cols, "r": r, "nsignal": nsignal,
            "rkins": rkins, "copied_rows": int(np.sum(src != np.arange(rows))), "miss_rate": 0.0}
    return Genotypes(out, rows, cols, ld, meta)
