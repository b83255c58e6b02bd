"""Seeded synthetic workloads shaped like the paper's 2D/3D manufactured-solution
tests (Example 1 and 2 of Section 6).  This module only produces plain numbers
(mesh sizes, partition cuts, parameters, time step, step count); it holds none
of the scheme's arithmetic and serves the library and the CPU oracle alike.

Random draws use SplitMix64 (Steele, Lea, Flood 2014): u = (x >> 11) 2^-53,
logU[a, b] = a (b/a)^u, integer shift s = (x mod 9) - 4.
"""

MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.state = seed & MASK

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next() >> 11) * 2.0 ** -53

    def log_uniform(self, a, b):
        return a * (b / a) ** self.uniform()


def unit_params():
    return dict(phi=[1.0] * 3, C=[1.0] * 3, k=[1.0] * 3, mu_tilde=1.0, sigma=1.0, sigma_star=1.0,
                rho=1.0, alpha=1.0, eta=1.0, nu=1.0)


def uniform_cuts(N, n):
    return [i * (N // n) for i in range(n + 1)]


def flat_cuts(cuts):
    """Cuts dict -> the ABI's flat list (porous-x, porous-y, conduit-x, conduit-y)."""
    return [v for key in ((0, 0), (0, 1), (1, 0), (1, 1)) for v in cuts[key]]


def config(name):
    """Workload dict: NH, refine, Nh, nsub, overlap, cuts ({(region, axis): list}),
    prm, dt, steps, dim, supported (2D only in this build)."""
    if name == "cfg1":
        NH, k, ns, ov = 4, 4, 4, 2
        prm, dt, steps = unit_params(), 0.1, 5
        cuts = None
    elif name == "cfg2":
        NH, k, ns, ov = 8, 8, 8, 4
        rng = SplitMix64(2)
        prm = unit_params()
        prm["nu"] = 1e-2
        kF, kf, km = (rng.log_uniform(1e-3, 1.0) for _ in range(3))
        sst = rng.log_uniform(0.1, 10.0)
        s = rng.log_uniform(0.1, 10.0)
        prm.update(k=[kF, kf, km], sigma_star=sst, sigma=s)
        dt, steps = 0.01, 100
        cuts = None
    elif name == "cfg3":
        NH, k, ns, ov = 16, 16, 16, 8
        N = NH * k
        rng = SplitMix64(3)
        cuts = {}
        for key in ((0, 0), (0, 1), (1, 0), (1, 1)):
            c = uniform_cuts(N, ns)
            for i in range(1, ns):
                c[i] += (rng.next() % 9) - 4
            cuts[key] = c
        prm = unit_params()
        nu = rng.log_uniform(1e-3, 1.0)
        kF, kf, km = (rng.log_uniform(1e-4, 1.0) for _ in range(3))
        sst = rng.log_uniform(0.1, 10.0)
        s = rng.log_uniform(0.1, 10.0)
        prm.update(nu=nu, k=[kF, kf, km], sigma_star=sst, sigma=s)
        dt, steps = 1e-3, 50
    elif name in ("cfg4", "cfg5"):
        return dict(name=name, dim=3, supported=False)
    else:
        raise KeyError(name)
    N = NH * k
    if cuts is None:
        cuts = {key: uniform_cuts(N, ns) for key in ((0, 0), (0, 1), (1, 0), (1, 1))}
    return dict(name=name, dim=2, supported=True, NH=NH, refine=k, Nh=N, nsub=(ns, ns), overlap=ov,
                cuts=cuts, prm=prm, dt=dt, steps=steps)


def ensemble_samples(n, seed=5):
    """n seeded parameter samples with the ensemble's ranges: nu logU[1e-3, 1],
    permeabilities k_F, k_f, k_m logU[1e-5, 1], exchange coefficients sigma*,
    sigma logU[0.01, 10] (draw order nu, k_F, k_f, k_m, sigma*, sigma per
    sample); the other parameters are 1."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(n):
        nu = rng.log_uniform(1e-3, 1.0)
        k = [rng.log_uniform(1e-5, 1.0) for _ in range(3)]
        sst = rng.log_uniform(0.01, 10.0)
        s = rng.log_uniform(0.01, 10.0)
        out.append(dict(unit_params(), nu=nu, k=k, sigma_star=sst, sigma=s))
    return out


def ensemble(nsamples=32, seed=5):
    """The parameter ensemble on the 2D geometry of cfg2 (H = 1/8, h = 1/64,
    8 x 8 subdomains per region, overlap 4 fine cells): nsamples seeded samples
    (ensemble_samples), dt = 0.01, 10 steps."""
    cfg = config("cfg2")
    return dict(cfg, name="ensemble", prm=None, samples=ensemble_samples(nsamples, seed), steps=10)


def shifted_small(seed=7):
    """Uneven cores at a size the oracle finishes in seconds: H = 1/4, h = 1/16,
    4 x 4 subdomains per region, overlap 2 fine cells, every interior cut of
    each (region, axis) shifted by (x mod 3) - 1 fine cells (SplitMix64, draw
    order porous x, porous y, conduit x, conduit y), non-unit parameters."""
    NH, k, ns, ov = 4, 4, 4, 2
    N = NH * k
    rng = SplitMix64(seed)
    cuts = {}
    for key in ((0, 0), (0, 1), (1, 0), (1, 1)):
        c = uniform_cuts(N, ns)
        for i in range(1, ns):
            c[i] += (rng.next() % 3) - 1
        cuts[key] = c
    prm = dict(unit_params(), nu=0.1, k=[0.5, 0.05, 0.01], sigma=3.0, sigma_star=0.3)
    return dict(name="shifted_small", dim=2, supported=True, NH=NH, refine=k, Nh=N, nsub=(ns, ns),
                overlap=ov, cuts=cuts, prm=prm, dt=0.02, steps=3)


def small(NH=2, refine=4, nsub=2, overlap=1, dt=0.05, prm=None):
    """A small custom 2D case for parity tests."""
    N = NH * refine
    return dict(name="small", dim=2, supported=True, NH=NH, refine=refine, Nh=N, nsub=(nsub, nsub),
                overlap=overlap, cuts={key: uniform_cuts(N, nsub) for key in ((0, 0), (0, 1), (1, 0), (1, 1))},
                prm=prm or unit_params(), dt=dt, steps=3)
