"""Seeded synthetic workloads shaped like the paper's Monte Carlo experiments.

This module only draws random numbers and lays them out; it contains none of
the estimator's arithmetic (no Fourier sums, no spreading, no weights), so both
the CPU oracle and the GPU library may consume what it produces.

Price model: correlated geometric Brownian motion stepped by Euler-Maruyama in
log space, S(t+h) = S(t) exp[(mu - sigma^2/2) h + sqrt(h) A Z] with A the
Cholesky factor of the covariance (the paper's GBM algorithm, appendix
"Algorithms"; SDE in Sec. 3).  Asynchrony is the paper's arrival-time
representation (Sec. 3): each asset observes the synchronous path at the
arrival times of its own Poisson process, taking the previous-tick price.

Parameters are "daily" and one second is 1/86400 day (Sec. 3.2 setting of the
accuracy experiments).  Every return delta_h = p(t_{h+1}) - p(t_h) is attached
to the left time t_h (Eq. for F(dp_i)(k), Sec. 2.2), so a series with n
observations carries n-1 events.

Output layout (CSR): ``offsets[S+1]`` int64, ``t[E]`` float64 (nondecreasing
within a series), ``dp[E]`` float64 or float32.  Series are grouped as G groups
of D consecutive assets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

SECONDS_PER_DAY = 86400.0


@dataclass
class Workload:
    name: str
    offsets: torch.Tensor          # int64 [S+1]
    t: torch.Tensor                # float64 [E]
    dp: torch.Tensor               # float64 or float32 [E]
    t0: float
    T: float
    G: int
    D: int
    Ns: list                       # sorted unique cutoffs
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def S(self) -> int:
        return self.offsets.numel() - 1

    @property
    def E(self) -> int:
        return int(self.offsets[-1])

    def to(self, device) -> "Workload":
        return Workload(self.name, self.offsets.to(device), self.t.to(device),
                        self.dp.to(device), self.t0, self.T, self.G, self.D,
                        list(self.Ns), self.seed, dict(self.meta))

    def series(self, s: int):
        a, b = int(self.offsets[s]), int(self.offsets[s + 1])
        return self.t[a:b], self.dp[a:b]

    def subset(self, idx) -> "Workload":
        """Series ``idx`` (list) as a new workload with G=1, D=len(idx)."""
        ts, ds, offs = [], [], [0]
        for s in idx:
            tt, dd = self.series(int(s))
            ts.append(tt)
            ds.append(dd)
            offs.append(offs[-1] + tt.numel())
        return Workload(self.name + "-subset", torch.tensor(offs, dtype=torch.int64),
                        torch.cat(ts), torch.cat(ds), self.t0, self.T, 1, len(idx),
                        list(self.Ns), self.seed, dict(self.meta))


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def logspace_int(nmax: int, count: int) -> list:
    """Unique integers round(logspace(0, log10 nmax, count)), ascending."""
    if nmax <= 1:
        return [1]
    vals = sorted({int(round(10 ** (i * math.log10(nmax) / (count - 1)))) for i in range(count)})
    return [v for v in vals if 1 <= v <= nmax]


def cov_from(sigma2, corr):
    s = torch.sqrt(torch.as_tensor(sigma2, dtype=torch.float64))
    c = torch.as_tensor(corr, dtype=torch.float64)
    return c * s[:, None] * s[None, :]


def gbm_log_increments(n_steps: int, mu, sigma2, corr, h: float, gen, device="cpu"):
    """Euler-Maruyama log increments of a correlated GBM on a uniform grid.

    Returns a (n_steps, D) float64 tensor of p(t_{k+1}) - p(t_k), step h (days).
    """
    mu = torch.as_tensor(mu, dtype=torch.float64, device=device)
    sigma2 = torch.as_tensor(sigma2, dtype=torch.float64, device=device)
    A = torch.linalg.cholesky(cov_from(sigma2.cpu(), torch.as_tensor(corr).cpu())).to(device)
    Z = torch.randn(n_steps, mu.numel(), generator=gen, dtype=torch.float64, device=device)
    return (mu - 0.5 * sigma2) * h + math.sqrt(h) * (Z @ A.T)


def poisson_times(rate: float, T: float, gen, device="cpu"):
    """Arrival times of a rate-``rate`` Poisson process on [0, T), float64."""
    mean = rate * T
    chunk = int(mean + 8.0 * math.sqrt(mean) + 16)
    out = []
    base = 0.0
    while True:
        e = torch.empty(chunk, dtype=torch.float64, device=device).exponential_(rate, generator=gen)
        c = base + torch.cumsum(e, 0)
        keep = c[c < T]
        out.append(keep)
        if keep.numel() < chunk:
            break
        base = float(c[-1])
    return torch.cat(out)


def _pack(name, series, t0, T, G, D, Ns, seed, dp_dtype, meta):
    offs = [0]
    for tt, _ in series:
        offs.append(offs[-1] + tt.numel())
    t = torch.cat([tt for tt, _ in series]).to(torch.float64)
    dp = torch.cat([dd for _, dd in series]).to(dp_dtype)
    return Workload(name, torch.tensor(offs, dtype=torch.int64, device=t.device), t, dp,
                    float(t0), float(T), G, D, Ns, seed, meta)


def _previous_tick(path, grid_h, times):
    """Observed log price at each time: the synchronous path at the last grid
    point at or before it (the arrival-time sampling of Sec. 3)."""
    idx = torch.clamp(torch.floor(times / grid_h).to(torch.int64), 0, path.shape[0] - 1)
    return path[idx]


# --------------------------------------------------------------------------------------
# Workloads.  Sizes and distributions follow the paper's experiments; the docstrings give
# the realised quantities.
# --------------------------------------------------------------------------------------

BIVARIATE = dict(mu=(0.01, 0.01), sigma2=(0.1, 0.2), rho=0.35, S0=100.0)


def bivariate_sync(n: int = 10_000, seed: int = 20200306, dp_dtype=torch.float64,
                   mu=BIVARIATE["mu"], sigma2=BIVARIATE["sigma2"], rho=BIVARIATE["rho"],
                   T_days: float = 1.0, device="cpu") -> Workload:
    """Tiny plain case: D=2 GBM, n synchronous equally spaced observations over
    one day (step T/n), times in days; N = n/2 (the synchronous Nyquist cutoff).
    Each asset carries n-1 returns at times t_h = h*T/n, h=0..n-2."""
    g = _gen(seed, "cpu")
    corr = [[1.0, rho], [rho, 1.0]]
    h = T_days / n
    inc = gbm_log_increments(n - 1, mu, sigma2, corr, h, g).to(device)
    times = torch.arange(n - 1, dtype=torch.float64, device=device) * h
    series = [(times.clone(), inc[:, i].clone()) for i in range(2)]
    true_cov = cov_from(sigma2, corr) * T_days
    return _pack("bivariate-sync", series, 0.0, T_days, 1, 2, [n // 2], seed, dp_dtype,
                 dict(true_cov=true_cov, n=n))


def bivariate_async(rates=(1 / 15, 1 / 30), T_sec: float = 28_800.0, seed: int = 20200307,
                    n_N: int = 40, dp_dtype=torch.float32, mu=BIVARIATE["mu"],
                    sigma2=BIVARIATE["sigma2"], rho=BIVARIATE["rho"], device="cpu") -> Workload:
    """Asynchronous bivariate: GBM on a 1 s grid over T_sec seconds sampled by
    independent Poisson arrivals (previous tick); cutoffs are the unique values of
    round(logspace(0, log10(n_min/2), n_N))."""
    g = _gen(seed, "cpu")
    corr = [[1.0, rho], [rho, 1.0]]
    n_grid = int(T_sec)
    inc = gbm_log_increments(n_grid, mu, sigma2, corr, 1.0 / SECONDS_PER_DAY, g)
    path = torch.cat([torch.zeros(1, 2, dtype=torch.float64), torch.cumsum(inc, 0)])
    series = []
    for i, r in enumerate(rates):
        tau = poisson_times(r, T_sec, g)
        p = _previous_tick(path[:, i], 1.0, tau)
        series.append((tau[:-1], p[1:] - p[:-1]))
    n_min = min(tt.numel() + 1 for tt, _ in series)
    Ns = logspace_int(max(1, n_min // 2), n_N)
    true_cov = cov_from(sigma2, corr) * (T_sec / SECONDS_PER_DAY)
    w = _pack("bivariate-async", series, 0.0, T_sec, 1, 2, Ns, seed, dp_dtype,
              dict(true_cov=true_cov, rates=list(rates)))
    return w.to(device)


def random_spd_corr(D: int, lo: float, hi: float, gen) -> torch.Tensor:
    """Symmetric matrix with unit diagonal and off-diagonals ~U(lo, hi), redrawn
    until it is positive definite (Cholesky succeeds)."""
    for _ in range(10_000):
        u = lo + (hi - lo) * torch.rand(D, D, generator=gen, dtype=torch.float64)
        c = torch.triu(u, 1)
        c = c + c.T + torch.eye(D, dtype=torch.float64)
        _, info = torch.linalg.cholesky_ex(c)
        if int(info) == 0:
            return c
    raise RuntimeError("could not draw an SPD correlation matrix")


def cross_section(D: int = 100, T_sec: float = 28_800.0, N: int = 5000, seed: int = 20200308,
                  rate_lo: float = 1 / 60, rate_hi: float = 1 / 2, factor_grid: float = 1e-3,
                  dp_dtype=torch.float32, device="cpu") -> Workload:
    """One-factor cross-section: loadings L_i~U(0.2,0.8) (corr_ij = L_i L_j),
    variances U(0.05,0.3) daily, mu=0.01; Poisson rates U(rate_lo, rate_hi)/s.
    The factor is a Brownian path on a ``factor_grid``-second grid observed by
    previous tick; idiosyncratic increments are exact at the event times."""
    g = _gen(seed, "cpu")
    L = 0.2 + 0.6 * torch.rand(D, generator=g, dtype=torch.float64)
    sig2 = 0.05 + 0.25 * torch.rand(D, generator=g, dtype=torch.float64)
    rates = rate_lo + (rate_hi - rate_lo) * torch.rand(D, generator=g, dtype=torch.float64)
    mu = 0.01
    n_f = int(round(T_sec / factor_grid))
    hf = factor_grid / SECONDS_PER_DAY
    F = torch.cat([torch.zeros(1, dtype=torch.float64),
                   torch.cumsum(math.sqrt(hf) * torch.randn(n_f, generator=g, dtype=torch.float64), 0)])
    series = []
    for i in range(D):
        tau = poisson_times(float(rates[i]), T_sec, g)
        tday = tau / SECONDS_PER_DAY
        dt = torch.diff(tday, prepend=torch.zeros(1, dtype=torch.float64))
        eps = torch.cumsum(torch.sqrt(dt) * torch.randn(tau.numel(), generator=g, dtype=torch.float64), 0)
        li = float(L[i])
        x = li * _previous_tick(F, factor_grid, tau) + math.sqrt(1 - li * li) * eps
        p = (mu - 0.5 * float(sig2[i])) * tday + math.sqrt(float(sig2[i])) * x
        series.append((tau[:-1], p[1:] - p[:-1]))
    corr = torch.outer(L, L)
    corr.fill_diagonal_(1.0)
    w = _pack("cross-section", series, 0.0, T_sec, 1, D, [N], seed, dp_dtype,
              dict(true_cov=cov_from(sig2, corr) * (T_sec / SECONDS_PER_DAY)))
    return w.to(device)


def epps_replicates(G: int = 1000, D: int = 10, T_sec: float = 28_800.0, Nmax: int = 2000,
                    n_N: int = 20, seed: int = 20200309, rate_lo: float = 1 / 30,
                    rate_hi: float = 1 / 5, dp_dtype=torch.float32, device="cpu") -> Workload:
    """Monte Carlo replicates: G independent D-asset GBMs (random SPD correlation
    with entries U(0.1,0.6), variances U(0.05,0.3)) on a 1 s grid over T_sec,
    each asset sampled by Poisson arrivals at a rate ~U(rate_lo, rate_hi)/s.
    Cutoffs: unique round(logspace(0, log10 Nmax, n_N))."""
    g = _gen(seed, device)
    gc = _gen(seed + 1, "cpu")
    corr = random_spd_corr(D, 0.1, 0.6, gc)
    sig2 = 0.05 + 0.25 * torch.rand(D, generator=gc, dtype=torch.float64)
    A = torch.linalg.cholesky(cov_from(sig2, corr)).to(device)
    drift = (0.01 - 0.5 * sig2).to(device)
    n_grid = int(T_sec)
    h = 1.0 / SECONDS_PER_DAY
    rates = rate_lo + (rate_hi - rate_lo) * torch.rand(G, D, generator=gc, dtype=torch.float64)
    # pad wide enough for the largest Poisson count with overwhelming probability
    nmax = int(rate_hi * T_sec + 10 * math.sqrt(rate_hi * T_sec) + 32)
    ts, ds, counts = [], [], []
    for r in range(G):
        Z = torch.randn(n_grid, D, generator=g, dtype=torch.float64, device=device)
        path = torch.cat([torch.zeros(1, D, dtype=torch.float64, device=device),
                          torch.cumsum(drift * h + math.sqrt(h) * (Z @ A.T), 0)])
        lam = rates[r].to(device)
        e = torch.empty(D, nmax, dtype=torch.float64, device=device).exponential_(1.0, generator=g)
        tau = torch.cumsum(e, 1) / lam[:, None]
        for i in range(D):
            ti = tau[i][tau[i] < T_sec]
            if ti.numel() == nmax:
                raise RuntimeError("Poisson padding exhausted")
            p = _previous_tick(path[:, i], 1.0, ti)
            ts.append(ti[:-1])
            ds.append(p[1:] - p[:-1])
            counts.append(ti.numel() - 1)
    offs = torch.zeros(G * D + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(torch.tensor(counts, dtype=torch.int64), 0)
    return Workload("epps-replicates", offs.to(device), torch.cat(ts), torch.cat(ds).to(dp_dtype),
                    0.0, T_sec, G, D, logspace_int(Nmax, n_N), seed,
                    dict(true_cov=cov_from(sig2, corr) * (T_sec / SECONDS_PER_DAY),
                         true_corr=corr, rates=rates))


def epps_pairs(G: int = 100, rho: float = 0.35, lam: float = 1 / 5, T_sec: float = 28_800.0,
               seed: int = 20200311, dp_dtype=torch.float32, device="cpu") -> Workload:
    """G replicates of a bivariate GBM (sigma^2 = (0.1, 0.2) daily, correlation
    rho, mu = 0.01) on a 1 s grid over T_sec, both assets sampled by independent
    Poisson arrivals of intensity lam per second (previous-tick prices): the
    setting of the Epps-effect model, Eq. Der:21."""
    g = _gen(seed, device)
    sig2 = torch.tensor([0.1, 0.2], dtype=torch.float64)
    corr = torch.tensor([[1.0, rho], [rho, 1.0]], dtype=torch.float64)
    A = torch.linalg.cholesky(cov_from(sig2, corr)).to(device)
    drift = (0.01 - 0.5 * sig2).to(device)
    n_grid = int(T_sec)
    h = 1.0 / SECONDS_PER_DAY
    nmax = int(lam * T_sec + 10 * math.sqrt(lam * T_sec) + 32)
    ts, ds, counts = [], [], []
    for r in range(G):
        Z = torch.randn(n_grid, 2, generator=g, dtype=torch.float64, device=device)
        path = torch.cat([torch.zeros(1, 2, dtype=torch.float64, device=device),
                          torch.cumsum(drift * h + math.sqrt(h) * (Z @ A.T), 0)])
        e = torch.empty(2, nmax, dtype=torch.float64, device=device).exponential_(1.0, generator=g)
        tau = torch.cumsum(e, 1) / lam
        for i in range(2):
            ti = tau[i][tau[i] < T_sec]
            if ti.numel() == nmax:
                raise RuntimeError("Poisson padding exhausted")
            p = _previous_tick(path[:, i], 1.0, ti)
            ts.append(ti[:-1])
            ds.append(p[1:] - p[:-1])
            counts.append(ti.numel() - 1)
    offs = torch.zeros(2 * G + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(torch.tensor(counts, dtype=torch.int64), 0)
    return Workload("epps-pairs", offs.to(device), torch.cat(ts), torch.cat(ds).to(dp_dtype), 0.0, T_sec, G, 2,
                    [1], seed, dict(rho=rho, lam=lam))


def missing_data(n: int = 10_000, keep: float = 0.6, seed: int = 20200312, dp_dtype=torch.float64) -> Workload:
    """The missing-data representation: the bivariate synchronous GBM on n equally
    spaced times over one day with each asset keeping a random fraction ``keep``
    of its observations (the paper down-samples by 40%); returns span the gaps."""
    w = bivariate_sync(n=n, seed=seed, dp_dtype=torch.float64)
    g = _gen(seed + 1, "cpu")
    series = []
    for s in range(2):
        tt, dd = w.series(s)
        logp = torch.cat([torch.zeros(1, dtype=torch.float64), torch.cumsum(dd, 0)])   # n observations
        times = torch.cat([tt, tt[-1:] + w.T / n])                                      # all n observation times
        mask = torch.rand(times.numel(), generator=g) < keep
        mask[0] = True
        mask[-1] = True
        tk, lk = times[mask], logp[mask]
        series.append((tk[:-1], lk[1:] - lk[:-1]))
    return _pack("missing-data", series, w.t0, w.T, 1, 2, [w.Ns[0]], seed, dp_dtype, dict(keep=keep))


def large_universe(D: int = 2000, n_lo: float = 1e4, n_hi: float = 1e6, N: int = 50_000,
                   T_sec: float = 28_800.0, n_factors: int = 3, factor_grid: float = 1e-3,
                   seed: int = 20200310, dp_dtype=torch.float32, device="cpu") -> Workload:
    """Large universe: D assets, 3-factor model with loadings B_if ~ N(0, 0.5^2)
    (corr = normalise(B B^T + I)), variances U(0.05,0.3) daily, mu = 0.01.
    Event counts are log-uniform in [n_lo, n_hi]; given its count, an asset's
    event times are the order statistics of that many uniforms on [0, T_sec)
    (a Poisson process conditioned on its count), drawn as normalised
    cumulative sums of exponentials.  Factors are Brownian paths on a
    ``factor_grid``-second grid observed by previous tick; idiosyncratic
    increments are exact at each event.  All assets are drawn at once with flat
    tensors on ``device``."""
    gc = _gen(seed, "cpu")
    g = _gen(seed + 1, device)
    B = 0.5 * torch.randn(D, n_factors, generator=gc, dtype=torch.float64)
    norm = torch.sqrt((B * B).sum(1) + 1.0)
    sig2 = 0.05 + 0.25 * torch.rand(D, generator=gc, dtype=torch.float64)
    logn = math.log(n_lo) + (math.log(n_hi) - math.log(n_lo)) * torch.rand(D, generator=gc, dtype=torch.float64)
    counts = torch.round(torch.exp(logn)).to(torch.int64)          # observations per asset
    n_f = int(round(T_sec / factor_grid))
    hf = factor_grid / SECONDS_PER_DAY
    F = torch.zeros(n_factors, n_f + 1, dtype=torch.float64, device=device)
    F[:, 1:] = torch.cumsum(math.sqrt(hf) * torch.randn(n_factors, n_f, generator=g, dtype=torch.float64,
                                                       device=device), 1)
    # observation times: asset i owns observations obs_off[i] .. obs_off[i+1]-1 and one
    # extra exponential that normalises its cumulative sum
    obs_off = torch.zeros(D + 1, dtype=torch.int64)
    obs_off[1:] = torch.cumsum(counts, 0)
    n_obs = int(obs_off[-1])
    asset = torch.repeat_interleave(torch.arange(D, device=device), (counts + 1).to(device))
    e = torch.empty(n_obs + D, dtype=torch.float64, device=device).exponential_(1.0, generator=g)
    c = torch.cumsum(e, 0)
    ext_off = (obs_off + torch.arange(D + 1)).to(device)            # offsets with the extra draw
    base = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), c[ext_off[1:-1] - 1]])
    total = c[ext_off[1:] - 1] - base                               # per-asset normaliser
    keep = torch.ones(n_obs + D, dtype=torch.bool, device=device)
    keep[ext_off[1:] - 1] = False                                   # drop each asset's extra draw
    a_obs = asset[keep]
    tau = T_sec * ((c[keep] - base[a_obs]) / total[a_obs])
    tau.clamp_(max=math.nextafter(T_sec, 0.0))
    tday = tau / SECONDS_PER_DAY
    # exact idiosyncratic Brownian motion at the observation times
    first = torch.zeros(n_obs, dtype=torch.bool, device=device)
    first[obs_off[:-1].to(device)] = True
    dtd = torch.where(first, tday, tday - torch.roll(tday, 1))
    z = torch.randn(n_obs, generator=g, dtype=torch.float64, device=device) * torch.sqrt(dtd)
    cz = torch.cumsum(z, 0)
    zbase = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), cz[obs_off[1:-1].to(device) - 1]])
    eps = cz - zbase[a_obs]
    Bd = (B / norm[:, None]).to(device)
    fidx = torch.clamp(torch.floor(tau / factor_grid).to(torch.int64), 0, n_f)
    x = (F[:, fidx] * Bd[a_obs].T).sum(0) + eps / norm.to(device)[a_obs]
    sd = torch.sqrt(sig2).to(device)[a_obs]
    p = (0.01 - 0.5 * sig2.to(device)[a_obs]) * tday + sd * x
    # returns attached to the left time; each asset's last observation carries none
    last = torch.zeros(n_obs, dtype=torch.bool, device=device)
    last[obs_off[1:].to(device) - 1] = True
    ret = torch.roll(p, -1) - p
    t = tau[~last].contiguous()
    dp = ret[~last].to(dp_dtype).contiguous()
    offs = torch.zeros(D + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(counts - 1, 0)
    corr = (B @ B.T + torch.eye(D, dtype=torch.float64)) / torch.outer(norm, norm)
    return Workload("large-universe", offs.to(device), t, dp, 0.0, T_sec, 1, D, [N], seed,
                    dict(true_cov=cov_from(sig2, corr) * (T_sec / SECONDS_PER_DAY), counts=counts))


def single_jump(u: float, delta: float, T: float = 1.0, dp_dtype=torch.float64) -> Workload:
    """One event of size delta at time u*T (the single-jump closed-form case)."""
    return Workload("single-jump", torch.tensor([0, 1], dtype=torch.int64),
                    torch.tensor([u * T], dtype=torch.float64), torch.tensor([delta], dtype=dp_dtype),
                    0.0, T, 1, 1, [1], 0, {})


def random_events(S: int, n_lo: int, n_hi: int, seed: int, T: float = 1.0,
                  dp_dtype=torch.float64, device="cpu", scale: float = 1e-3) -> Workload:
    """S series with uniform random sorted times on [0, T) and N(0, scale^2)
    strengths; counts uniform in [n_lo, n_hi] (n_lo may be 0: empty series)."""
    g = _gen(seed, "cpu")
    counts = torch.randint(n_lo, n_hi + 1, (S,), generator=g)
    ts, ds = [], []
    for i in range(S):
        n = int(counts[i])
        tt, _ = torch.sort(T * torch.rand(n, generator=g, dtype=torch.float64))
        ts.append(tt)
        ds.append(scale * torch.randn(n, generator=g, dtype=torch.float64))
    offs = torch.zeros(S + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(counts, 0)
    w = Workload("random-events", offs, torch.cat(ts) if ts else torch.zeros(0, dtype=torch.float64),
                 (torch.cat(ds) if ds else torch.zeros(0, dtype=torch.float64)).to(dp_dtype),
                 0.0, T, 1, S, [1], seed, {})
    return w.to(device)
