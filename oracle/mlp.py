"""FP64 numpy reference of the learned moving prior -- TEST INFRASTRUCTURE.

Section 2.1 of the paper computes moving priors from the weight distribution over
integrals of motion (or approximately conserved quantities) such as E, L, Lz.
The learned form reads that as a smooth function fitted to the weights:
ln what(E, L, Lz) = g(u) + const, with g a multilayer perceptron 3 -> 64 -> 64 -> 1
(tanh hidden units), features u = (2 (E - Emin)/(Emax - Emin) - 1, 2 L/Lc(E) - 1, Lz/L),
trained on the current weights with the mean squared error of g(u_i) - ln w_i and
Adam (Kingma & Ba 2015, Algorithm 1).  Priors are rescaled so that sum what = sum w.

Flat parameter vector (4481 values): W1[64,3], b1[64], W2[64,64], b2[64], W3[1,64], b3[1],
row-major, output index first.
"""
import numpy as np

H = 64
SIZES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def forward(theta, u):
    """u [B, 3] -> g [B] (and the hidden activations)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    h1 = np.tanh(u @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    g = h2 @ p["W3"].T + p["b3"]
    return g[:, 0], h1, h2


def loss(theta, u, t):
    g, _, _ = forward(theta, u)
    return float(np.mean((g - t) ** 2))


def loss_grad(theta, u, t):
    """Loss and its gradient with respect to the flat parameter vector (backpropagation)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    g, h1, h2 = forward(theta, u)
    B = u.shape[0]
    dg = 2.0 * (g - t) / B                      # [B]
    gW3 = dg[None, :] @ h2                      # [1, H]
    gb3 = np.array([dg.sum()])
    da2 = (dg[:, None] @ p["W3"]) * (1.0 - h2 * h2)   # [B, H]
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (1.0 - h1 * h1)
    gW1 = da1.T @ u
    gb1 = da1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.mean((g - t) ** 2)), grad


def adam(theta, grad, m, v, t, lr, b1, b2, eps):
    """One Adam step (t counts from 1); returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(E, L, Lz, Lc, Emin, Emax):
    u0 = 2.0 * (E - Emin) / (Emax - Emin) - 1.0
    u1 = np.where(Lc > 0, 2.0 * L / np.where(Lc > 0, Lc, 1.0) - 1.0, -1.0)
    u2 = np.where(L > 0, Lz / np.where(L > 0, L, 1.0), 0.0)
    return np.stack([u0, u1, u2], axis=1)


def priors(theta, u, w):
    """what_i = s exp(g(u_i)) with s such that sum what = sum w."""
    g, _, _ = forward(theta, u)
    g = g - g.max()
    e = np.exp(g)
    return e * (w.sum() / e.sum())


def judge(w, what_mlp, what_hist):
    """w-weighted mean |ln what_mlp - ln what_hist| (fallback test)."""
    return float(np.sum(w * np.abs(np.log(what_mlp) - np.log(what_hist))) / np.sum(w))


class LearnedPrior:
    """The learned moving prior of one model over a run (reading of section 2.1):
    every `period` steps, at refresh q = n / period, before the step's update,
      1. a sample of `subset` particle indices, Philox4x32-10 counter (k/4, q, 0, 0)
         under key (seed, 0), index = (word * N) >> 32 (the oracle's subset());
      2. Adam on the sample in consecutive minibatches of `batch`, with the
         moments and the step count carried over from earlier refreshes, on the
         mean squared error of g(u_i) - ln w_i at the current weights;
      3. what_i = s exp(g(u_i)) over all particles, sum what = sum w;
      4. the judge against the histogram prior on the same cells (the mean weight
         of each particle's cell): above `fallback` the histogram prior is used.
    The priors are held until the next refresh."""

    def __init__(self, theta0, lr, beta1, beta2, eps, seed, subset, batch, fallback):
        self.theta = np.asarray(theta0, dtype=np.float64).copy()
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.seed, self.subset, self.batch, self.fallback = seed, subset, batch, fallback
        self.last_judge = None
        self.used_fallback = None

    def refresh(self, q, idx, u, w, what_hist):
        """One refresh: idx the sample (subset indices), u [N, 3] features, w the
        weights, what_hist the histogram prior; returns the priors."""
        tgt = np.log(w)
        for b0 in range(0, self.subset, self.batch):
            sl = idx[b0:b0 + self.batch]
            _, g = loss_grad(self.theta, u[sl], tgt[sl])
            self.t += 1
            self.theta, self.m, self.v = adam(self.theta, g, self.m, self.v, self.t, self.lr, self.beta1,
                                              self.beta2, self.eps)
        what = priors(self.theta, u, w)
        self.last_judge = judge(w, what, what_hist)
        self.used_fallback = self.last_judge > self.fallback
        return what_hist.copy() if self.used_fallback else what


def run(model, lp, prior_cfg, nsteps, subset_fn):
    """Run an oracle model (oracle.Model) nsteps with the learned prior lp:
    refreshes at the steps n with n % period == 0.  subset_fn(seed, q, count, N)
    gives the sample indices.  Returns the per-step statistics rows."""
    P = int(prior_cfg.get("period", 1))
    Emin, Emax = model.Erange
    rows = []
    for _ in range(nsteps):
        n = model.step_index
        if n % P == 0:
            E, L, Lz, Lc = model.integrals()
            u = features(E, L, Lz, Lc, Emin, Emax)
            what_hist = model.prior_means()[0]
            idx = subset_fn(lp.seed, n // P, lp.subset, u.shape[0])
            model.set_what(lp.refresh(n // P, idx, u, model.w, what_hist))
        rows.append(model.run(1)[0])
    return np.array(rows)
