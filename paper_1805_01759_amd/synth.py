"""Seeded synthetic TomoSAR stacks (inputs only; none of the solver's arithmetic).

Both the GPU path's tests/benchmark and the FP64 oracle draw their inputs from
here.  The imaging model is Eq. (2) / Eq. (5) of arXiv 1805.01759 with no
motion term: a pixel's measurement vector is
    g_n = sum_k gamma_k exp(-j 2 pi xi_n s_k) + eps_n,   xi_n = 2 b_n / (lambda_w r),
and A[n, l] = exp(-j 2 pi xi_n s_l) samples the same phase on a uniform
elevation grid s_l.  (The paper writes exp(+j...); the sign convention only
conjugates the problem.)  Scatterer amplitudes are CN(0, 1), the noise is
CN(0, sigma^2) per acquisition with sigma^2 = 10^(-SNR/10), and the
regularisation weight is lambda = sigma sqrt(2 N ln L).

Randomness: numpy Philox.  Key = 1805_01759 + config id (+ stack id); every
block of ``BLOCK`` pixels has its own counter offset, so any pixel range can be
regenerated alone and gives the same values as the full stack.  Everything is
generated in float64; ``to_device_dtypes`` rounds to complex64/float32 once,
and the oracle upcasts those same rounded values.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os

import numpy as np

KEY = 1805_01759
BLOCK = 4096
WAVELENGTH = 0.031  # m (X band)
RANGE = 7.0e5       # m


@dataclasses.dataclass
class Geometry:
    n: int
    l: int
    baselines: np.ndarray  # (N,) metres
    xi: np.ndarray         # (N,) cycles per metre
    s: np.ndarray          # (L,) elevation grid, metres
    A: np.ndarray          # (N, L) complex128

    @property
    def rayleigh(self) -> float:
        """Elevation resolution from the realised aperture, lambda_w r / (2 (b_max - b_min))."""
        return WAVELENGTH * RANGE / (2.0 * float(self.baselines.max() - self.baselines.min()))


@dataclasses.dataclass
class Spec:
    cfg: int
    n: int
    l: int
    p: int
    bmax: float
    s_lo: float
    s_hi: float
    model: str          # "c1" | "c2" | "c4" | "c5"
    snr_db: float | None = 10.0


SPECS = {
    1: Spec(1, 15, 101, 1024, 250.0, -50.0, 50.0, "c1", 10.0),
    2: Spec(2, 25, 256, 1 << 20, 300.0, -60.0, 60.0, "c2", None),
    4: Spec(4, 50, 512, 1 << 22, 300.0, -60.0, 60.0, "c4", 10.0),
    5: Spec(5, 25, 256, 1 << 18, 300.0, -60.0, 60.0, "c5", 10.0),
}


def _gen(cfg: int, stack: int, stream: int, block: int) -> np.random.Generator:
    key = ((KEY + cfg) << 40) | (stack << 8) | stream
    return np.random.Generator(np.random.Philox(key=key, counter=[0, 0, block, 0]))


def make_geometry(cfg: int, n: int, l: int, bmax: float, s_lo: float, s_hi: float,
                  stack: int = 0) -> Geometry:
    g = _gen(cfg, stack, 0, 0)
    b = g.uniform(-bmax, bmax, size=n)
    xi = 2.0 * b / (WAVELENGTH * RANGE)
    s = np.linspace(s_lo, s_hi, l)
    A = np.exp(-2j * np.pi * np.outer(xi, s))
    return Geometry(n, l, b, xi, s, A)


def steering(xi: np.ndarray, s: np.ndarray) -> np.ndarray:
    """exp(-j 2 pi xi_n s) for an array of elevations s (shape (..., ) -> (..., N))."""
    return np.exp(-2j * np.pi * np.multiply.outer(s, xi))


def _cn(g, size, var=1.0):
    return (g.standard_normal(size) + 1j * g.standard_normal(size)) * math.sqrt(var / 2.0)


def _block_pixels(spec: Spec, geom: Geometry, block: int, count: int, stack: int):
    """Pixels [block*BLOCK, block*BLOCK + count) of one stack."""
    g = _gen(spec.cfg, stack, 1, block)
    n, l = geom.n, geom.l
    lo, hi = float(geom.s[0]), float(geom.s[-1])
    # two scatterer slots per pixel; unused slots carry zero amplitude
    amp = _cn(g, (count, 2))
    elev = g.uniform(lo, hi, size=(count, 2))
    xtrue_idx = np.full((count, 2), -1, np.int64)
    if spec.model == "c2":
        k = g.choice(3, size=count, p=[0.3, 0.5, 0.2])
    else:
        k = g.integers(0, 3, size=count)
    if spec.model == "c4":
        pair = g.uniform(size=count) < 0.4
        kappa = g.uniform(0.3, 1.0, size=count)
        ds = kappa * geom.rayleigh
        mid = g.uniform(lo + ds / 2.0, hi - ds / 2.0)
        zero_phase = g.uniform(size=count) < 0.1
        e2 = np.stack([mid - ds / 2.0, mid + ds / 2.0], axis=1)
        elev = np.where(pair[:, None], e2, elev)
        k = np.where(pair, 2, k)
        a1 = amp[:, 1]
        same = np.abs(a1) * np.exp(1j * np.angle(amp[:, 0]))
        amp[:, 1] = np.where(pair & zero_phase, same, a1)
    if spec.model == "c5":
        # on-grid scatterers, so that the true profile is an L-vector
        idx = g.integers(0, l, size=(count, 2))
        elev = geom.s[idx]
        xtrue_idx = idx
    amp = amp * (np.arange(2)[None, :] < k[:, None])
    if spec.snr_db is None:
        snr = g.uniform(0.0, 20.0, size=count)
    else:
        snr = np.full(count, spec.snr_db)
    sigma2 = 10.0 ** (-snr / 10.0)
    noise = _cn(g, (count, n)) * np.sqrt(sigma2)[:, None]
    B = np.einsum("pk,pkn->pn", amp, steering(geom.xi, elev)) + noise
    lam = np.sqrt(sigma2) * math.sqrt(2.0 * n * math.log(l))
    meta = {"k": k, "elev": elev, "amp": amp, "snr_db": snr, "xtrue_idx": xtrue_idx}
    return B, lam, meta


def _map_blocks(fn, blocks):
    """fn over pixel blocks; blocks draw from their own counters, so running them
    on several threads gives the same values as one after another."""
    if len(blocks) < 8:
        return [fn(b) for b in blocks]
    workers = min(16, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, blocks))


def make_pixels(spec: Spec, geom: Geometry, p0: int = 0, p1: int | None = None,
                stack: int = 0, with_meta: bool = False):
    """B (P, N) complex128 and lambda (P,) float64 for pixels [p0, p1)."""
    p1 = spec.p if p1 is None else p1
    Bs, lams, metas = [], [], []
    b0, b1 = p0 // BLOCK, (p1 - 1) // BLOCK
    blocks = list(range(b0, b1 + 1))
    outs = _map_blocks(lambda blk: _block_pixels(spec, geom, blk, min(BLOCK, spec.p - blk * BLOCK),
                                                 stack), blocks)
    for blk, (B, lam, meta) in zip(blocks, outs):
        start = blk * BLOCK
        cnt = min(BLOCK, spec.p - start)
        lo, hi = max(p0 - start, 0), min(p1 - start, cnt)
        Bs.append(B[lo:hi])
        lams.append(lam[lo:hi])
        if with_meta:
            metas.append({k: v[lo:hi] for k, v in meta.items()})
    B = np.concatenate(Bs) if Bs else np.zeros((0, geom.n), np.complex128)
    lam = np.concatenate(lams) if lams else np.zeros(0)
    if not with_meta:
        return B, lam
    meta = {k: np.concatenate([m[k] for m in metas]) for k in metas[0]} if metas else {}
    return B, lam, meta


def make_config(cfg: int, p0: int = 0, p1: int | None = None, with_meta: bool = False,
                p_override: int | None = None):
    """Geometry and pixels of one single-stack configuration (1, 2, 4 or 5)."""
    spec = dataclasses.replace(SPECS[cfg])
    if p_override is not None:
        spec.p = p_override
    geom = make_geometry(cfg, spec.n, spec.l, spec.bmax, spec.s_lo, spec.s_hi)
    out = make_pixels(spec, geom, p0, p1, with_meta=with_meta)
    return (spec, geom) + tuple(out)


def xtrue(spec: Spec, geom: Geometry, meta) -> np.ndarray:
    """On-grid true profile (configuration 5): X_true[p, idx] = amplitude."""
    p = meta["amp"].shape[0]
    X = np.zeros((p, geom.l), np.complex128)
    for slot in range(2):
        np.add.at(X, (np.arange(p), meta["xtrue_idx"][:, slot]), meta["amp"][:, slot])
    return X


# ------------------------------------------------------------ batched stacks

@dataclasses.dataclass
class StackSpec:
    stack: int
    n: int
    l: int
    p: int


def batched_specs(num_stacks: int = 64, scale: float = 1.0) -> list[StackSpec]:
    """Uneven stacks: N ~ U{10..100}, L ~ U{64..1024}, P log-uniform in [1e3, 2.56e5].

    ``scale`` multiplies every pixel count (for reduced test sizes)."""
    g = _gen(3, 0, 2, 0)
    out = []
    for i in range(num_stacks):
        n = int(g.integers(10, 101))
        l = int(g.integers(64, 1025))
        p = int(round(math.exp(g.uniform(math.log(1e3), math.log(2.56e5)))))
        out.append(StackSpec(i, n, l, max(1, int(round(p * scale)))))
    return out


def make_batched_stack(ss: StackSpec, p0: int = 0, p1: int | None = None):
    spec = Spec(3, ss.n, ss.l, ss.p, 250.0, -50.0, 50.0, "c1", 10.0)
    geom = make_geometry(3, ss.n, ss.l, 250.0, -50.0, 50.0, stack=ss.stack + 1)
    B, lam = make_pixels(spec, geom, p0, p1, stack=ss.stack + 1)
    return spec, geom, B, lam


def to_device_dtypes(A, B, lam):
    """Round once to the GPU's storage types (complex64 / float32)."""
    return (np.ascontiguousarray(A, np.complex64), np.ascontiguousarray(B, np.complex64),
            np.ascontiguousarray(lam, np.float32))


def uniform_draws(count: int, seed: int = 0) -> np.ndarray:
    """`count` uniform float64 draws in [0, 1) (the random numbers a randomized
    block method consumes, one per iteration), from the same keyed Philox stream
    family as the stacks."""
    g = np.random.Generator(np.random.Philox(key=KEY + 9000 + seed))
    return g.random(count)


# ------------------------------------------------ multicomponent (D-TomoSAR) stacks
#
# Eqs. (3)-(4): with linear motion the phase of a scatterer at elevation s moving
# at velocity v (line of sight) is 2 pi (xi_n s + eta_n v), eta_n = 2 t_n / lambda_w
# for acquisition times t_n; the unknown becomes a profile over the elevation x
# velocity grid and A gains one column per grid point.  Column c = i + Ls j holds
# exp(-j 2 pi (xi_n s_i + eta_n v_j)) (elevation the fast index), i.e. A is the
# column-wise Kronecker product of the elevation and velocity steering matrices.
# A seasonal component (Eq. (4) with the temporal base function sin(2 pi t), period
# one year) adds zeta_n = 2 sin(2 pi t_n) / lambda_w and a third axis of seasonal
# amplitudes a_k: column i + Ls j + Ls Lv k holds exp(-j 2 pi (xi_n s_i + eta_n v_j +
# zeta_n a_k)); with one seasonal level at a = 0 it is the elevation x velocity grid.

@dataclasses.dataclass
class MotionSpec:
    cfg: int
    n: int
    ls: int               # elevation bins
    lv: int               # velocity bins
    p: int
    bmax: float = 300.0   # baselines U[-bmax, bmax] m
    years: float = 3.0    # acquisition times U[0, years]
    s_lo: float = -60.0
    s_hi: float = 60.0
    v_lo: float = -0.04   # m / year
    v_hi: float = 0.04
    la: int = 1           # seasonal-amplitude bins (1: no seasonal axis)
    a_lo: float = 0.0     # m
    a_hi: float = 0.0

    @property
    def l(self) -> int:
        return self.ls * self.lv * self.la


@dataclasses.dataclass
class MotionGeometry:
    n: int
    ls: int
    lv: int
    baselines: np.ndarray  # (N,) m
    times: np.ndarray      # (N,) years, ascending
    xi: np.ndarray         # (N,) cycles per metre of elevation
    eta: np.ndarray        # (N,) cycles per (metre / year) of velocity
    s: np.ndarray          # (Ls,) elevation grid, m
    v: np.ndarray          # (Lv,) velocity grid, m / year
    A: np.ndarray          # (N, Ls Lv La) complex128
    la: int = 1
    zeta: np.ndarray | None = None  # (N,) cycles per metre of seasonal amplitude
    a: np.ndarray | None = None     # (La,) seasonal-amplitude grid, m

    @property
    def l(self) -> int:
        return self.ls * self.lv * self.la


MOTION_SPECS = {
    # N = 50 acquisitions over three years; 32 elevation x 16 velocity bins (L = 512)
    6: MotionSpec(6, 50, 32, 16, 1 << 19),
    # the same stack on a finer elevation grid: 64 x 16 = 1024 bins
    7: MotionSpec(7, 50, 64, 16, 1 << 16),
    # elevation x velocity x seasonal amplitude (up to 10 mm): 32 x 16 x 8 = 4096 bins
    10: MotionSpec(10, 50, 32, 16, 1 << 15, la=8, a_lo=-0.01, a_hi=0.01),
}


def motion_steering(geom: MotionGeometry, s: np.ndarray, v: np.ndarray, a: np.ndarray | None = None) -> np.ndarray:
    """exp(-j 2 pi (xi_n s + eta_n v + zeta_n a)) for arrays s, v (, a) of one shape
    (..., ) -> (..., N); without a seasonal axis the last term is absent."""
    ph = np.multiply.outer(s, geom.xi) + np.multiply.outer(v, geom.eta)
    if a is not None and geom.zeta is not None:
        ph = ph + np.multiply.outer(a, geom.zeta)
    return np.exp(-2j * np.pi * ph)


def make_motion_geometry(spec: MotionSpec, stack: int = 0) -> MotionGeometry:
    g = _gen(spec.cfg, stack, 0, 0)
    b = g.uniform(-spec.bmax, spec.bmax, size=spec.n)
    t = np.sort(g.uniform(0.0, spec.years, size=spec.n))
    xi = 2.0 * b / (WAVELENGTH * RANGE)
    eta = 2.0 * t / WAVELENGTH
    s = np.linspace(spec.s_lo, spec.s_hi, spec.ls)
    v = np.linspace(spec.v_lo, spec.v_hi, spec.lv)
    geom = MotionGeometry(spec.n, spec.ls, spec.lv, b, t, xi, eta, s, v, None)
    if spec.la == 1:
        ss, vv = np.meshgrid(s, v)            # (Lv, Ls): column c = i + Ls j
        geom.A = np.ascontiguousarray(motion_steering(geom, ss.ravel(), vv.ravel()).T)
        return geom
    geom.la = spec.la
    geom.zeta = 2.0 * np.sin(2.0 * np.pi * t) / WAVELENGTH
    geom.a = np.linspace(spec.a_lo, spec.a_hi, spec.la)
    aa, vv, ss = np.meshgrid(geom.a, v, s, indexing="ij")  # (La, Lv, Ls): c = i + Ls j + Ls Lv k
    geom.A = np.ascontiguousarray(motion_steering(geom, ss.ravel(), vv.ravel(), aa.ravel()).T)
    return geom


def _motion_block_pixels(spec: MotionSpec, geom: MotionGeometry, block: int, count: int, stack: int):
    """Pixels [block*BLOCK, block*BLOCK + count): 0/1/2 scatterers (0.3/0.5/0.2)
    at off-grid (elevation, velocity), CN(0, 1) amplitudes, SNR U[0, 20] dB."""
    g = _gen(spec.cfg, stack, 1, block)
    amp = _cn(g, (count, 2))
    elev = g.uniform(spec.s_lo, spec.s_hi, size=(count, 2))
    vel = g.uniform(spec.v_lo, spec.v_hi, size=(count, 2))
    k = g.choice(3, size=count, p=[0.3, 0.5, 0.2])
    amp = amp * (np.arange(2)[None, :] < k[:, None])
    snr = g.uniform(0.0, 20.0, size=count)
    sigma2 = 10.0 ** (-snr / 10.0)
    noise = _cn(g, (count, spec.n)) * np.sqrt(sigma2)[:, None]
    # seasonal amplitudes (drawn last, so that stacks without the axis keep their draws)
    seas = g.uniform(spec.a_lo, spec.a_hi, size=(count, 2)) if spec.la > 1 else None
    B = np.einsum("pk,pkn->pn", amp, motion_steering(geom, elev, vel, seas)) + noise
    lam = np.sqrt(sigma2) * math.sqrt(2.0 * spec.n * math.log(spec.l))
    meta = {"k": k, "elev": elev, "vel": vel, "amp": amp, "snr_db": snr}
    if seas is not None:
        meta["seas"] = seas
    return B, lam, meta


def make_motion_config(cfg: int, p0: int = 0, p1: int | None = None, with_meta: bool = False,
                       p_override: int | None = None):
    """Spec, geometry, B (P, N) complex128 and lambda (P,) of pixels [p0, p1) of a
    multicomponent stack (configuration 6, 7 or, with the seasonal axis, 10)."""
    spec = dataclasses.replace(MOTION_SPECS[cfg])
    if p_override is not None:
        spec.p = p_override
    geom = make_motion_geometry(spec)
    p1 = spec.p if p1 is None else p1
    Bs, lams, metas = [], [], []
    blocks = list(range(p0 // BLOCK, (p1 - 1) // BLOCK + 1 if p1 > p0 else p0 // BLOCK))
    outs = _map_blocks(lambda blk: _motion_block_pixels(spec, geom, blk,
                                                        min(BLOCK, spec.p - blk * BLOCK), 0), blocks)
    for blk, (B, lam, meta) in zip(blocks, outs):
        start = blk * BLOCK
        cnt = min(BLOCK, spec.p - start)
        lo, hi = max(p0 - start, 0), min(p1 - start, cnt)
        Bs.append(B[lo:hi])
        lams.append(lam[lo:hi])
        metas.append({k: v[lo:hi] for k, v in meta.items()})
    B = np.concatenate(Bs) if Bs else np.zeros((0, spec.n), np.complex128)
    lam = np.concatenate(lams) if lams else np.zeros(0)
    if not with_meta:
        return spec, geom, B, lam
    meta = {k: np.concatenate([m[k] for m in metas]) for k in metas[0]} if metas else {}
    return spec, geom, B, lam, meta


# ------------------------------------------- super-resolution (two close scatterers)
#
# The double-scatterer simulations: N = 29 acquisitions over the elevation
# aperture of the paper's real stack (269.5 m), two scatterers of unit
# amplitude placed symmetrically about s = 0 at a distance kappa rho_s
# (rho_s = lambda_w r / (2 Delta b), the Rayleigh resolution) and complex
# Gaussian noise at a per-scatterer SNR.  Two sets of cases:
#   "profiles"  (the reconstructed profiles): kappa 1.2, 0.8, 0.4, 0.2 at SNR
#               10, 3, 0 dB; the phase difference is not stated there, so it is
#               drawn uniformly per realisation;
#   "detection" (detection rate against kappa): SNR 2 dB and 7 dB for both
#               scatterers, phase difference 0 (the worst case), kappa 0.2 to
#               1.2 in steps of 0.2.
# Realisations differ in noise (and phase); the baselines are one fixed draw
# that spans the whole aperture.

SUPERRES_N = 29
SUPERRES_APERTURE = 269.5     # m
SUPERRES_L = 256
SUPERRES_S = (-80.0, 80.0)    # elevation grid, m
SUPERRES_CFG = 8
SUPERRES_CASES = ([("profiles", k, snr) for k in (1.2, 0.8, 0.4, 0.2) for snr in (10.0, 3.0, 0.0)] +
                  [("detection", k, snr) for snr in (2.0, 7.0) for k in (0.2, 0.4, 0.6, 0.8, 1.0, 1.2)])


def make_superres_geometry() -> Geometry:
    g = _gen(SUPERRES_CFG, 0, 0, 0)
    half = SUPERRES_APERTURE / 2.0
    inner = g.uniform(-half, half, size=SUPERRES_N - 2)
    b = np.sort(np.concatenate([[-half, half], inner]))
    xi = 2.0 * b / (WAVELENGTH * RANGE)
    s = np.linspace(SUPERRES_S[0], SUPERRES_S[1], SUPERRES_L)
    return Geometry(SUPERRES_N, SUPERRES_L, b, xi, s, np.exp(-2j * np.pi * np.outer(xi, s)))


def make_superres(realisations: int, cases=None, r0: int = 0):
    """Geometry, B (P, N) complex128, lambda (P,) and per-pixel metadata for
    realisations [r0, r0 + realisations) of every case (set, kappa, SNR dB);
    pixels run case by case, realisations inner-most.  Realisation r of case c
    draws from counter r of its own stream, so any range regenerates alone."""
    geom = make_superres_geometry()
    rho = geom.rayleigh
    cases = SUPERRES_CASES if cases is None else cases
    out = {k: [] for k in ("B", "lam", "case", "kappa", "snr_db", "s1", "s2", "dphi")}
    for c, (kind, kappa, snr) in enumerate(cases):
        s1, s2 = -kappa * rho / 2.0, kappa * rho / 2.0
        a1 = steering(geom.xi, np.array([s1]))[0]
        a2 = steering(geom.xi, np.array([s2]))[0]
        sigma2 = 10.0 ** (-snr / 10.0)
        Bc, dph = [], []
        for r in range(r0, r0 + realisations):
            g = _gen(SUPERRES_CFG, c + 1, 1, r)
            dphi = g.uniform(0.0, 2.0 * math.pi) if kind == "profiles" else 0.0
            Bc.append(a1 + np.exp(1j * dphi) * a2 + _cn(g, geom.n) * math.sqrt(sigma2))
            dph.append(dphi)
        out["B"].append(np.array(Bc))
        out["dphi"].append(np.array(dph))
        lam = math.sqrt(sigma2) * math.sqrt(2.0 * geom.n * math.log(geom.l))
        for key, v in (("lam", lam), ("case", c), ("kappa", kappa), ("snr_db", snr), ("s1", s1), ("s2", s2)):
            out[key].append(np.full(realisations, v))
    B = np.concatenate(out.pop("B"))
    lam = np.concatenate(out.pop("lam"))
    meta = {k: np.concatenate(v) for k, v in out.items()}
    return geom, B, lam, meta
