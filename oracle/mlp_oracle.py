"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

Plain numpy: `layers` ReLU layers, a linear layer to `rank` coefficients and
a linear output layer, mean squared error, backpropagation and Adam, written
from their definitions.  The flat parameter layout (per layer W [in x out]
then b [out]) is the interface the GPU network also uses; nothing else is
shared.  The gradient is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


class MLPRef:
    def __init__(self, in_dim, hidden, layers, rank, out_dim):
        self.dims = [in_dim] + [hidden] * layers + [rank, out_dim]
        self.relu = [True] * layers + [False, False]
        self.shapes = []
        off = 0
        for a, b in zip(self.dims[:-1], self.dims[1:]):
            self.shapes.append((off, a, b))
            off += a * b + b
        self.nparam = off

    def unpack(self, p):
        out = []
        for off, a, b in self.shapes:
            W = p[off:off + a * b].reshape(a, b)
            bias = p[off + a * b:off + a * b + b]
            out.append((W, bias))
        return out

    def forward(self, p, X, mu, sigma):
        """Returns the activations [standardized input, layer 1 out, ...]."""
        acts = [(np.asarray(X, np.float64) - mu) / sigma]
        for (W, b), r in zip(self.unpack(np.asarray(p, np.float64)), self.relu):
            h = acts[-1] @ W + b
            if r:
                h = np.maximum(h, 0.0)
            acts.append(h)
        return acts

    def loss(self, p, X, Zs, mu, sigma):
        Z = self.forward(p, X, mu, sigma)[-1]
        return float(np.mean((Z - Zs) ** 2))

    def loss_grad(self, p, X, Zs, mu, sigma):
        """Mean squared error over all B*out_dim entries and its gradient."""
        p = np.asarray(p, np.float64)
        acts = self.forward(p, X, mu, sigma)
        Z = acts[-1]
        d = Z - Zs
        loss = float(np.mean(d * d))
        g = np.zeros(self.nparam)
        dY = 2.0 * d / d.size
        params = self.unpack(p)
        for li in range(len(params) - 1, -1, -1):
            off, a, b = self.shapes[li]
            if self.relu[li]:
                dY = dY * (acts[li + 1] > 0)
            g[off:off + a * b] = (acts[li].T @ dY).ravel()
            g[off + a * b:off + a * b + b] = dY.sum(axis=0)
            dY = dY @ params[li][0].T
        return loss, g

    @staticmethod
    def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step (t counts from 1); returns new (p, m, v)."""
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        return p - lr * mh / (np.sqrt(vh) + eps), m, v
