"""Seeded synthetic workloads for the QEM E-step.

This module is the single source of inputs shared by the HIP path and the
CPU oracle.  It describes each model's structure (latent nodes, plates,
observation families, the initial proposal) and draws ground-truth latents and
raw observations from the generative model with numpy's PCG64 generator.

It deliberately holds none of the method's arithmetic: no log-densities,
no sufficient statistics, no importance weights, no moments.  Each consumer
computes those itself from the raw arrays returned here.

Model families (the hierarchies the paper's experiments are built from, with
the sizes of the five benchmark configurations as defaults):

* ``normal_normal``   2-level Gaussian: mu ~ N(0,1); z_i ~ N(mu, 1); x_ij ~ N(z_i, 0.25).
* ``nested_gaussian`` 3-level Gaussian in R^d: mu ~ N(0,I); schools s ~ N(mu, I);
                      classes c ~ N(s, 0.25 I); students x ~ N(c, I).
* ``chain``           G independent random walks z_0 ~ N(0,1),
                      z_t ~ N(0.9 z_{t-1}, 0.09), x_t ~ N(z_t, 0.25).
* ``gamma_poisson``   alpha, beta ~ Gamma(2,1); lambda_i ~ Gamma(alpha, beta);
                      y_ij ~ Poisson(lambda_i).
* ``logistic``        beta ~ N(0, I_D); log sigma ~ N(0,1); b_i ~ N(0, sigma^2);
                      y_ij ~ Bernoulli(sigmoid(x_ij . beta + b_i)), x_ij ~ N(0, I_D).
* ``occupancy``       site occupancy z_i ~ Bernoulli(sigmoid(psi)), repeated
                      detections y_ij ~ Bernoulli(p z_i) (discrete latents).
* ``ar_regions``      region levels under a global mean, an AR(1) series per
                      region around its level (chains under a sampled parent).
* ``dirichlet_categorical``  group proportions pi_i ~ Dirichlet(s), categorical
                      draws y_ij ~ Categorical(pi_i).
* ``mixture``         mixture weights pi ~ Dirichlet(1), memberships c_i ~
                      Categorical(pi), observations y_ij ~ N(mu_{c_i}, var).

Conventions: N(mean, variance); Gamma(shape, rate).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Node", "Obs", "Model",
    "normal_normal", "nested_gaussian", "chain", "gamma_poisson", "logistic",
    "occupancy", "ar_regions", "dirichlet_categorical", "mixture",
    "tiny_tree", "CONFIGS", "make",
]


@dataclass
class Node:
    """One latent variable node, replicated over a plate of ``n`` instances.

    prior kinds
      ``normal``          z ~ N(a * z_parent + b, var) per dimension (no parent: N(b, var)).
                          With ``chain_len`` T > 1 the ``n`` instances form n/T series
                          laid out [series, T]; step 0 ~ N(init_b, init_var) and step t
                          ~ N(a z_{t-1} + b, var) within its series.  A chain with a
                          (scalar) parent takes one parent instance beta per series:
                          step 0 ~ N(beta + init_b, init_var), step t ~ N(a z_{t-1}
                          + (1 - a) beta + b, var).
      ``gamma``           z ~ Gamma(shape, rate) with constant shape and rate.
      ``gamma_parents``   z ~ Gamma(parent0, parent1) (shape node, rate node).
      ``normal_logscale`` z ~ N(0, exp(parent0)^2).
      ``bernoulli_logit`` z in {0, 1} ~ Bernoulli(sigmoid(a * z_parent + b)) (no parent:
                          sigmoid(b)); for ``bernoulli`` proposals, q0 = (p, 1).
      ``dirichlet``       z on the simplex of dim = C components ~ Dir(shape, ..., shape);
                          for ``dirichlet`` proposals, q0 = (alpha, 1): Dir(alpha, ..., alpha).
      ``categorical``     z one-hot over dim = C categories; P(c) = pi_c of a Dirichlet parent
                          (no parent: 1 / C); for ``categorical`` proposals q0 = (p, 1): every
                          category starts with weight p.
    """
    name: str
    n: int
    dim: int
    qfamily: str                      # "gauss" | "gamma" | "gamma_ef" | "bernoulli" | "dirichlet" | "categorical"
    prior: str                        # see above
    parents: Tuple[int, ...] = ()
    parent_index: Optional[np.ndarray] = None   # int32 [n] -> instance of parents[0]
    a: float = 1.0
    b: float = 0.0
    var: float = 1.0
    shape: float = 2.0
    rate: float = 1.0
    chain_len: int = 0
    init_b: float = 0.0
    init_var: float = 1.0
    q0: Tuple[float, float] = (0.0, 1.0)  # initial Q: (mean, var) or (shape, rate)


@dataclass
class Obs:
    """Observations attached to the instances of one latent node.

    kinds
      ``gauss``           x[n, J, dim] ~ N(z, var)
      ``poisson``         y[n, J] ~ Poisson(z)
      ``bernoulli_logit`` y[n, J] ~ Bernoulli(sigmoid(cov[n, J, :] . z_coef + z)),
                          with ``coef`` the node holding the coefficient vector.
      ``detection``       y[n, J] in {0, 1} ~ Bernoulli(var * z), z a Bernoulli latent
                          (``var`` is the detection probability).
      ``categorical``     y[n, J] in {0, .., dim - 1} ~ Categorical(z), z a Dirichlet latent.
      ``gauss_mixture``   y[n, J] ~ N(mu_c, var), c the category of a categorical latent z,
                          ``cov`` the component means mu [C].
    """
    node: int
    kind: str
    x: np.ndarray
    var: float = 1.0
    coef: int = -1
    cov: Optional[np.ndarray] = None


@dataclass
class Model:
    name: str
    nodes: List[Node]
    obs: List[Obs]
    truth: List[np.ndarray] = field(default_factory=list)
    K: int = 8
    iters: int = 20
    lam: float = 0.3

    def n_latent_instances(self) -> int:
        return int(sum(nd.n for nd in self.nodes))


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([20250311, int(seed)]))


def normal_normal(seed: int = 0, n_groups: int = 8, n_obs: int = 4, K: int = 8) -> Model:
    rng = _rng(seed)
    mu = rng.normal(0.0, 1.0, size=(1, 1))
    z = mu[0, 0] + rng.normal(0.0, 1.0, size=(n_groups, 1))
    x = z[:, None, :] + 0.5 * rng.normal(size=(n_groups, n_obs, 1))
    nodes = [
        Node("mu", 1, 1, "gauss", "normal", a=0.0, b=0.0, var=1.0),
        Node("z", n_groups, 1, "gauss", "normal", parents=(0,),
             parent_index=np.zeros(n_groups, np.int32), a=1.0, b=0.0, var=1.0),
    ]
    return Model("normal_normal", nodes, [Obs(1, "gauss", x, var=0.25)], [mu, z], K=K, iters=20, lam=0.3)


def nested_gaussian(seed: int = 0, n_schools: int = 256, n_classes: int = 32,
                    n_students: int = 16, dim: int = 4, K: int = 64) -> Model:
    rng = _rng(seed)
    mu = rng.normal(size=(1, dim))
    s = mu + rng.normal(size=(n_schools, dim))
    sidx = np.repeat(np.arange(n_schools, dtype=np.int32), n_classes)
    c = s[sidx] + 0.5 * rng.normal(size=(n_schools * n_classes, dim))
    x = c[:, None, :] + rng.normal(size=(n_schools * n_classes, n_students, dim))
    nodes = [
        Node("mu", 1, dim, "gauss", "normal", a=0.0, b=0.0, var=1.0),
        Node("school", n_schools, dim, "gauss", "normal", parents=(0,),
             parent_index=np.zeros(n_schools, np.int32), a=1.0, var=1.0),
        Node("class", n_schools * n_classes, dim, "gauss", "normal", parents=(1,),
             parent_index=sidx, a=1.0, var=0.25),
    ]
    return Model("nested_gaussian", nodes, [Obs(2, "gauss", x, var=1.0)], [mu, s, c],
                 K=K, iters=100, lam=0.3)


def chain(seed: int = 0, n_series: int = 1024, T: int = 64, K: int = 256,
          a: float = 0.9, var: float = 0.09, obs_var: float = 0.25) -> Model:
    rng = _rng(seed)
    z = np.empty((n_series, T))
    z[:, 0] = rng.normal(size=n_series)
    for t in range(1, T):
        z[:, t] = a * z[:, t - 1] + np.sqrt(var) * rng.normal(size=n_series)
    x = z + np.sqrt(obs_var) * rng.normal(size=(n_series, T))
    nodes = [Node("z", n_series * T, 1, "gauss", "normal", a=a, b=0.0, var=var,
                  chain_len=T, init_b=0.0, init_var=1.0)]
    return Model("chain", nodes, [Obs(0, "gauss", x.reshape(n_series * T, 1, 1), var=obs_var)],
                 [z.reshape(-1, 1)], K=K, iters=50, lam=0.3)


def gamma_poisson(seed: int = 0, n_groups: int = 2048, n_obs: int = 64, K: int = 128,
                  qfamily: str = "gamma") -> Model:
    """qfamily "gamma" (moment-matched M-step) or "gamma_ef" (the
    exponential-family M-step on (E z, E log z)) for all three latents."""
    rng = _rng(seed)
    alpha = rng.gamma(2.0, 1.0)
    beta = rng.gamma(2.0, 1.0)
    lam = rng.gamma(alpha, 1.0 / beta, size=n_groups)
    y = rng.poisson(lam[:, None], size=(n_groups, n_obs)).astype(np.float64)
    nodes = [
        Node("alpha", 1, 1, qfamily, "gamma", shape=2.0, rate=1.0, q0=(2.0, 1.0)),
        Node("beta", 1, 1, qfamily, "gamma", shape=2.0, rate=1.0, q0=(2.0, 1.0)),
        Node("lambda", n_groups, 1, qfamily, "gamma_parents", parents=(0, 1),
             parent_index=np.zeros(n_groups, np.int32), q0=(2.0, 1.0)),
    ]
    return Model("gamma_poisson", nodes, [Obs(2, "poisson", y)],
                 [np.array([[alpha]]), np.array([[beta]]), lam[:, None]], K=K, iters=100, lam=0.3)


def mixture(seed: int = 0, n_groups: int = 2048, C: int = 4, n_obs: int = 10, var: float = 1.0,
            K: int = 64) -> Model:
    """A Gaussian mixture with sampled weights: pi ~ Dir(1, ..., 1) over C
    components, memberships z_i ~ Categorical(pi), y_ij ~ N(mu_{z_i}, var)
    with known means mu = -3, ..., 3 evenly spaced.  Memberships start
    uniform, the weights at Dir(1, ..., 1)."""
    rng = _rng(seed)
    pi = rng.dirichlet(np.ones(C))
    z = rng.choice(C, size=n_groups, p=pi)
    mu = np.linspace(-3.0, 3.0, C)
    y = mu[z][:, None] + np.sqrt(var) * rng.normal(size=(n_groups, n_obs))
    nodes = [Node("pi", 1, C, "dirichlet", "dirichlet", shape=1.0, q0=(1.0, 1.0)),
             Node("z", n_groups, C, "categorical", "categorical", parents=(0,),
                  parent_index=np.zeros(n_groups, np.int32), q0=(1.0 / C, 1.0))]
    return Model("mixture", nodes, [Obs(1, "gauss_mixture", y, var=var, cov=mu.copy())],
                 [pi[None], np.eye(C)[z]], K=K, iters=50, lam=0.3)


def dirichlet_categorical(seed: int = 0, n_groups: int = 4096, C: int = 4, n_obs: int = 20, shape: float = 1.0,
                          K: int = 64) -> Model:
    """Category probabilities per group p_i ~ Dir(shape, ..., shape) over C
    categories, y_ij ~ Categorical(p_i), j < n_obs (C = 2: Beta-Bernoulli);
    the Dirichlet proposal starts at Dir(1, ..., 1).  The exact posterior of
    each group is Dir(shape + counts_i)."""
    rng = _rng(seed)
    p = rng.dirichlet(np.full(C, shape), size=n_groups)
    y = np.stack([rng.choice(C, size=n_obs, p=p[i]) for i in range(n_groups)]).astype(np.float64)
    nodes = [Node("p", n_groups, C, "dirichlet", "dirichlet", shape=shape, q0=(1.0, 1.0))]
    return Model("dirichlet_categorical", nodes, [Obs(0, "categorical", y)], [p], K=K, iters=50, lam=0.3)


def logistic(seed: int = 0, n_groups: int = 8192, n_obs: int = 50, D: int = 8, K: int = 64) -> Model:
    rng = _rng(seed)
    beta = rng.normal(size=(1, D))
    logsig = rng.normal(size=(1, 1))
    b = np.exp(logsig[0, 0]) * rng.normal(size=(n_groups, 1))
    cov = rng.normal(size=(n_groups, n_obs, D))
    eta = cov @ beta[0] + b
    y = (rng.uniform(size=eta.shape) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    nodes = [
        Node("beta", 1, D, "gauss", "normal", a=0.0, b=0.0, var=1.0),
        Node("logsigma", 1, 1, "gauss", "normal", a=0.0, b=0.0, var=1.0),
        Node("b", n_groups, 1, "gauss", "normal_logscale", parents=(1,),
             parent_index=np.zeros(n_groups, np.int32)),
    ]
    return Model("logistic", nodes, [Obs(2, "bernoulli_logit", y, coef=0, cov=cov)],
                 [beta, logsig, b], K=K, iters=250, lam=0.3)


def tiny_tree(seed: int = 0, K: int = 3) -> Model:
    """A 3-level Gaussian with 1 school x 2 classes (brute-force sized)."""
    m = nested_gaussian(seed, n_schools=1, n_classes=2, n_students=3, dim=2, K=K)
    m.name = "tiny_tree"
    return m


#: The five benchmark configurations, by name.
CONFIGS = {
    "c1_normal_normal": lambda seed=0: normal_normal(seed),
    "c2_nested_gaussian": lambda seed=0: nested_gaussian(seed),
    "c3_chain": lambda seed=0: chain(seed),
    "c4_gamma_poisson": lambda seed=0: gamma_poisson(seed),
    "c5_logistic": lambda seed=0: logistic(seed),
}


def make(name: str, seed: int = 0, **kw) -> Model:
    builders = {
        "normal_normal": normal_normal, "nested_gaussian": nested_gaussian, "chain": chain,
        "gamma_poisson": gamma_poisson, "logistic": logistic, "tiny_tree": tiny_tree, "occupancy": occupancy,
        "dirichlet_categorical": dirichlet_categorical, "mixture": mixture,
        "ar_regions": ar_regions,
    }
    if name in CONFIGS and not kw:
        return CONFIGS[name](seed)
    return builders[name](seed, **kw)


def occupancy(seed: int = 0, n_sites: int = 14400, n_visits: int = 5, p_det: float = 0.6,
              K: int = 30) -> Model:
    """Occupancy with imperfect detection (the shape of the paper's occupancy
    model, with its covariates collapsed into one occupancy logit): a global
    logit psi ~ N(0, 1.5^2), site occupancy z_i ~ Bernoulli(sigmoid(psi)),
    and n_visits detections per site y_ir ~ Bernoulli(p_det z_i).  Default
    size: 12 x 6 x 200 site-level latents, 5 visits, K = 30."""
    rng = _rng(seed)
    psi = rng.normal(0.0, 1.5)
    z = (rng.uniform(size=n_sites) < 1.0 / (1.0 + np.exp(-psi))).astype(np.float64)
    y = (rng.uniform(size=(n_sites, n_visits)) < p_det * z[:, None]).astype(np.float64)
    nodes = [
        Node("logit_psi", 1, 1, "gauss", "normal", a=0.0, b=0.0, var=2.25, q0=(0.0, 1.0)),
        Node("z", n_sites, 1, "bernoulli", "bernoulli_logit", parents=(0,),
             parent_index=np.zeros(n_sites, np.int32), a=1.0, b=0.0, q0=(0.5, 1.0)),
    ]
    return Model("occupancy", nodes, [Obs(1, "detection", y, var=p_det)],
                 [np.array([[psi]]), z[:, None]], K=K, iters=100, lam=0.3)


def ar_regions(seed: int = 0, n_regions: int = 92, T: int = 109, K: int = 64, a: float = 0.8,
               var: float = 0.1, obs_var: float = 0.25) -> Model:
    """AR(1) chains under K-sampled parents (the shape of the paper's Covid
    model: regions x days, with Gaussian observations standing in for its
    counts): mu ~ N(0, 1); region levels beta_r ~ N(mu, 0.5); per region a
    chain x_{r,0} ~ N(beta_r, 0.3), x_{r,t} ~ N(a x_{r,t-1} + (1 - a) beta_r,
    var); y_{r,t} ~ N(x_{r,t}, obs_var)."""
    rng = _rng(seed)
    mu = rng.normal()
    beta = mu + np.sqrt(0.5) * rng.normal(size=n_regions)
    x = np.empty((n_regions, T))
    x[:, 0] = beta + np.sqrt(0.3) * rng.normal(size=n_regions)
    for t in range(1, T):
        x[:, t] = a * x[:, t - 1] + (1.0 - a) * beta + np.sqrt(var) * rng.normal(size=n_regions)
    y = x.reshape(-1, 1, 1) + np.sqrt(obs_var) * rng.normal(size=(n_regions * T, 1, 1))
    nodes = [
        Node("mu", 1, 1, "gauss", "normal", a=0.0, b=0.0, var=1.0),
        Node("beta", n_regions, 1, "gauss", "normal", parents=(0,),
             parent_index=np.zeros(n_regions, np.int32), a=1.0, b=0.0, var=0.5),
        Node("x", n_regions * T, 1, "gauss", "normal", parents=(1,),
             parent_index=np.repeat(np.arange(n_regions, dtype=np.int32), T), a=a, b=0.0, var=var,
             chain_len=T, init_b=0.0, init_var=0.3),
    ]
    return Model("ar_regions", nodes, [Obs(2, "gauss", y, var=obs_var)],
                 [np.array([[mu]]), beta[:, None], x.reshape(-1, 1)], K=K, iters=100, lam=0.3)
