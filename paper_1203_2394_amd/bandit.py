"""Automatic choice of the state decomposition (Section 3, Fig. 5): the
Hedge and Exp3 bandits over K actions, here the sampling orders of the two
state blocks (action 1: x first, action 2: z first; Section 4.3).

Host-side control logic: a few scalar updates per time step over the
per-step rewards of filters that run on the GPU.

Reward (Section 4.3): r_t = alpha / (alpha + eps_t^2), eps_t the difference
between the observation y_t and the one-step-ahead predicted observation of
the chosen action's filter (the library's predicted observation,
dpf_set_prediction); 0 < r <= 1.

Hedge (Fig. 5, top) with memory parameter eta: at time t it chooses action i
with probability p_i(t) proportional to exp(eta G_i(t-1)), receives the whole
reward vector r(t) and sets G_i(t) = G_i(t-1) + r_i(t) for every i.

Exp3 (Fig. 5, bottom) with exploration gamma in (0, 1]: takes p(t) from its
Hedge, draws i_t from p^_j = (1 - gamma) p_j + gamma / K, receives only
r_{i_t}(t), and feeds Hedge the simulated vector r^_j = r_{i_t} / p^_{i_t}
for j = i_t and 0 otherwise.

Probabilities are formed with the largest exponent subtracted first (the
same distribution; no overflow once the cumulative gains grow large).
Actions are drawn by inverse CDF from caller-supplied uniforms, or from a
seeded NumPy PCG64 stream.
"""
import numpy as np


def reward(eps, alpha=1e-3):
    """alpha / (alpha + eps^2), elementwise."""
    eps = np.asarray(eps, dtype=np.float64)
    return alpha / (alpha + eps * eps)


def _draw(p, u):
    """Inverse-CDF draw: the first index whose cumulative probability
    exceeds u (u in [0, 1))."""
    c = np.cumsum(p)
    return int(min(np.searchsorted(c, u * c[-1], side="right"), len(p) - 1))


class Hedge:
    """Hedge(eta) over K actions."""

    def __init__(self, K, eta):
        if K < 1 or not eta > 0:
            raise ValueError("need K >= 1 and eta > 0")
        self.K = int(K)
        self.eta = float(eta)
        self.G = np.zeros(self.K)

    def probs(self):
        e = self.eta * self.G
        w = np.exp(e - e.max())
        return w / w.sum()

    def choose(self, u):
        return _draw(self.probs(), u)

    def update(self, r):
        r = np.asarray(r, dtype=np.float64)
        if r.shape != (self.K,):
            raise ValueError("reward vector of %d actions expected" % self.K)
        self.G = self.G + r


class Exp3:
    """Exp3(gamma, eta) over K actions (Hedge as its subroutine)."""

    def __init__(self, K, eta, gamma):
        if not 0.0 < gamma <= 1.0:
            raise ValueError("gamma must lie in (0, 1]")
        self.hedge = Hedge(K, eta)
        self.K = self.hedge.K
        self.gamma = float(gamma)

    def probs(self):
        """p^(t) = (1 - gamma) p(t) + gamma / K."""
        return (1.0 - self.gamma) * self.hedge.probs() + self.gamma / self.K

    def choose(self, u):
        return _draw(self.probs(), u)

    def update(self, i, r):
        """Feed the reward r of the chosen action i (probabilities of the
        same time step, i.e. before this update)."""
        ph = self.probs()
        rhat = np.zeros(self.K)
        rhat[i] = float(r) / ph[i]
        self.hedge.update(rhat)


def run_hedge(rewards, eta, uniforms):
    """Hedge over a reward sequence rewards [T][K] (every action's reward is
    observed, full information).  uniforms [T] pick the actions.  Returns
    (actions [T], probabilities [T][K] used at each step)."""
    R = np.asarray(rewards, dtype=np.float64)
    T, K = R.shape
    h = Hedge(K, eta)
    acts = np.empty(T, dtype=np.int64)
    P = np.empty((T, K))
    for t in range(T):
        P[t] = h.probs()
        acts[t] = _draw(P[t], float(uniforms[t]))
        h.update(R[t])
    return acts, P


def run_exp3(rewards, eta, gamma, uniforms):
    """Exp3 over a reward sequence rewards [T][K] of which only the chosen
    action's entry is used at each step.  uniforms [T] pick the actions.
    Returns (actions [T], Hedge probabilities p [T][K], mixed p^ [T][K])."""
    R = np.asarray(rewards, dtype=np.float64)
    T, K = R.shape
    e = Exp3(K, eta, gamma)
    acts = np.empty(T, dtype=np.int64)
    P = np.empty((T, K))
    Ph = np.empty((T, K))
    for t in range(T):
        P[t] = e.hedge.probs()
        Ph[t] = e.probs()
        i = _draw(Ph[t], float(uniforms[t]))
        acts[t] = i
        e.update(i, R[t, i])
    return acts, P, Ph


def uniforms(seed, T):
    """T uniforms in [0, 1) from a seeded PCG64 stream."""
    return np.random.Generator(np.random.PCG64(seed)).random(T)
