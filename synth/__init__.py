"""Seeded synthetic workloads for clustered multi-task compressive sensing.

Shared by the tests, the benchmark and the oracle checks; holds none of the method's arithmetic,
only the generative recipe of the data (Eq. (cmtcs) with Gaussian sensing matrices) and the
initial alpha draw of Alg. 2.

Recipe (all seeds fixed and recorded):
  * true clusters are contiguous blocks of tasks; cluster g draws one support S_g of size
    ``sparsity`` uniformly without replacement from {0..D-1}; task t draws its own N(0, 1) values
    on the support of its cluster;
  * Phi_t has i.i.d. N(0, 1/N_t) entries, stored float32, row-major [N_t][D]; all tasks are
    stacked in one [sum N_t][D] array with row offsets;
  * y_t = Phi_t z_t + sigma * N(0, I), stored float32;  beta = 1 / sigma^2;  pi uniform;
  * with ``support_diff`` = f >= 0 (two groups; the first experiment of Sec. 4): the groups share
    round((1 - f) * sparsity) support entries and draw the rest disjointly, so f = 0 gives one
    common support and f = 1 disjoint ones;
  * alpha^0 ~ Uniform(0, 1) i.i.d. per (c, d) (Alg. 2, initialisation), rounded to float32 so that
    every consumer sees identical values; zeros are redrawn.
"""

from dataclasses import dataclass, field
import numpy as np

DATA_SEED = 2310
INIT_SEED = 420
PROBE_SEED = 1


@dataclass
class Config:
    name: str
    T: int
    C: int
    D: int
    N: object              # int; (lo, hi) for N_t ~ Uniform{lo..hi}; or a list of T values
    sparsity: int
    groups: int            # number of true clusters (contiguous task blocks)
    K: int = 32
    fixed_iters: int = 0   # > 0: exactly this many CG steps
    tol: float = 1e-6
    max_iters: int = 200
    n_em: int = 1
    sigma: float = 0.01
    support_diff: float = -1.0   # >= 0: fraction f of the support that differs between 2 groups


CONFIGS = {
    # plain method, FP64, tiny: checked against exact dense EM
    "tiny": Config("tiny", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16, fixed_iters=64, n_em=20),
    # plain FP32 GPU path
    "fp32": Config("fp32", T=32, C=4, D=1024, N=256, sparsity=32, groups=4, K=32, n_em=30),
    # precision form (headline shape)
    "prec": Config("prec", T=64, C=4, D=4096, N=1024, sparsity=64, groups=4, K=32, n_em=1),
    # batching form: ragged N_t
    "batch": Config("batch", T=256, C=8, D=2048, N=(128, 2048), sparsity=48, groups=8, K=32, n_em=1),
    # differentiation form
    "diff": Config("diff", T=16, C=2, D=2048, N=512, sparsity=40, groups=2, K=0, n_em=1),
}


@dataclass
class Workload:
    cfg: Config
    Phi: np.ndarray            # [sum N_t][D] float32
    row_off: np.ndarray        # [T+1] int64
    y: np.ndarray              # [sum N_t] float32
    z: np.ndarray              # [T][D] float64 true signals
    labels: np.ndarray         # [T] true cluster of each task
    alpha0: np.ndarray         # [C][D] float32-representable values (float64 array)
    beta: float
    log_pi: np.ndarray         # [C]
    extra: dict = field(default_factory=dict)

    @property
    def T(self):
        return self.cfg.T

    def phi(self, t):
        return self.Phi[self.row_off[t]:self.row_off[t + 1]]

    def y_t(self, t):
        return self.y[self.row_off[t]:self.row_off[t + 1]]

    def phi_list(self):
        return [self.phi(t) for t in range(self.T)]

    def y_list(self):
        return [self.y_t(t) for t in range(self.T)]


def draw_alpha0(C, D, seed=INIT_SEED):
    rng = np.random.default_rng(seed)
    a = rng.random((C, D)).astype(np.float32)
    while (a == 0).any():
        z = a == 0
        a[z] = rng.random(int(z.sum())).astype(np.float32)
    return a.astype(np.float64)


def make(cfg, data_seed=DATA_SEED, init_seed=INIT_SEED, **over):
    """Build the workload of ``cfg`` (a Config or a name in CONFIGS); ``over`` replaces fields."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if over:
        cfg = Config(**{**cfg.__dict__, **over})
    rng = np.random.default_rng(data_seed)
    T, D = cfg.T, cfg.D
    if isinstance(cfg.N, list) and len(cfg.N) == T:
        Ns = np.asarray(cfg.N, dtype=np.int64)
    elif isinstance(cfg.N, (tuple, list)):
        Ns = rng.integers(cfg.N[0], cfg.N[1] + 1, size=T)
    else:
        Ns = np.full(T, int(cfg.N))
    row_off = np.zeros(T + 1, np.int64)
    row_off[1:] = np.cumsum(Ns)
    per = -(-T // cfg.groups)
    labels = np.minimum(np.arange(T) // per, cfg.groups - 1)
    if cfg.support_diff < 0:
        supports = [rng.choice(D, size=cfg.sparsity, replace=False) for _ in range(cfg.groups)]
    else:
        assert cfg.groups == 2 and 0.0 <= cfg.support_diff <= 1.0 and 2 * cfg.sparsity <= D
        n_sh = int(round((1.0 - cfg.support_diff) * cfg.sparsity))
        pick = rng.choice(D, size=2 * cfg.sparsity - n_sh, replace=False)
        own = cfg.sparsity - n_sh
        supports = [np.concatenate([pick[:n_sh], pick[n_sh:n_sh + own]]),
                    np.concatenate([pick[:n_sh], pick[n_sh + own:]])]
    Phi = np.empty((int(row_off[-1]), D), np.float32)
    y = np.empty(int(row_off[-1]), np.float32)
    z = np.zeros((T, D))
    for t in range(T):
        n = int(Ns[t])
        blk = rng.standard_normal((n, D), dtype=np.float32)
        blk *= np.float32(1.0 / np.sqrt(max(n, 1)))
        Phi[row_off[t]:row_off[t + 1]] = blk
        z[t, supports[labels[t]]] = rng.standard_normal(cfg.sparsity)
        y[row_off[t]:row_off[t + 1]] = (blk.astype(np.float64) @ z[t]
                                        + cfg.sigma * rng.standard_normal(n)).astype(np.float32)
    return Workload(cfg=cfg, Phi=Phi, row_off=row_off, y=y, z=z, labels=labels,
                    alpha0=draw_alpha0(cfg.C, D, init_seed), beta=1.0 / cfg.sigma ** 2,
                    log_pi=np.full(cfg.C, -np.log(cfg.C)), extra=dict(supports=supports))


def hadamard(m):
    """Sylvester-Hadamard matrix of order 2^m (entries +-1, H H^T = 2^m I)."""
    H = np.ones((1, 1))
    for _ in range(m):
        H = np.block([[H, H], [H, -H]])
    return H


# ------------------------------------------------------------------------------------------
# Partial-Fourier sensing (the experiments of Sec. 4): Phi_t = Omega_t F with F the unitary D x D
# DFT and Omega_t a random subset of N_t = D/4 of its rows; the complex measurements are
# y_t = Omega_t F z_t + sigma (e1 + i e2), e1, e2 ~ N(0, I), stored as float32 (re, im) pairs;
# the real model sees them stacked as [Re y_t; Im y_t] against [Re(Omega_t F); Im(Omega_t F)].
# Signals, clusters and alpha^0 follow the same recipe as above; sigma = 0.05 as in Sec. 4 and
# 5% of the entries of each signal are non-zero.

FOURIER_CONFIGS = {
    # small case for parity tests
    "fourier-small": Config("fourier-small", T=4, C=2, D=256, N=64, sparsity=13, groups=2, K=16,
                            sigma=0.05),
    # the metric's task, cluster, probe and length sizes with the paper's sensing
    "fourier": Config("fourier", T=64, C=4, D=4096, N=1024, sparsity=205, groups=4, K=32,
                      sigma=0.05),
}


@dataclass
class FourierWorkload:
    cfg: Config
    freq: np.ndarray           # [sum N_t] int32 selected frequencies, task t in row_off[t]:[t+1]
    row_off: np.ndarray        # [T+1] int64 prefix sums of N_t (complex measurements)
    yc: np.ndarray             # [sum N_t][2] float32 (re, im) measurements
    z: np.ndarray              # [T][D] float64 true signals
    labels: np.ndarray
    alpha0: np.ndarray
    beta: float
    log_pi: np.ndarray

    @property
    def T(self):
        return self.cfg.T

    def freq_t(self, t):
        return self.freq[self.row_off[t]:self.row_off[t + 1]]

    def yc_t(self, t):
        v = self.yc[self.row_off[t]:self.row_off[t + 1]].astype(np.float64)
        return v[:, 0] + 1j * v[:, 1]


def make_fourier(cfg, data_seed=DATA_SEED, init_seed=INIT_SEED, **over):
    if isinstance(cfg, str):
        cfg = FOURIER_CONFIGS[cfg]
    if over:
        cfg = Config(**{**cfg.__dict__, **over})
    rng = np.random.default_rng(data_seed)
    T, D = cfg.T, cfg.D
    Ns = np.full(T, int(cfg.N)) if not isinstance(cfg.N, (list, tuple)) else np.asarray(cfg.N)
    row_off = np.zeros(T + 1, np.int64)
    row_off[1:] = np.cumsum(Ns)
    per = -(-T // cfg.groups)
    labels = np.minimum(np.arange(T) // per, cfg.groups - 1)
    supports = [rng.choice(D, size=cfg.sparsity, replace=False) for _ in range(cfg.groups)]
    freq = np.empty(int(row_off[-1]), np.int32)
    yc = np.empty((int(row_off[-1]), 2), np.float32)
    z = np.zeros((T, D))
    for t in range(T):
        n = int(Ns[t])
        f = np.sort(rng.choice(D, size=n, replace=False))
        z[t, supports[labels[t]]] = rng.standard_normal(cfg.sparsity)
        Fz = np.fft.fft(z[t], norm="ortho")[f]
        noise = cfg.sigma * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        v = Fz + noise
        freq[row_off[t]:row_off[t + 1]] = f
        yc[row_off[t]:row_off[t + 1], 0] = v.real
        yc[row_off[t]:row_off[t + 1], 1] = v.imag
    return FourierWorkload(cfg=cfg, freq=freq, row_off=row_off, yc=yc, z=z, labels=labels,
                           alpha0=draw_alpha0(cfg.C, D, init_seed), beta=1.0 / cfg.sigma ** 2,
                           log_pi=np.full(cfg.C, -np.log(cfg.C)))
