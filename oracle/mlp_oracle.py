"""Plain FP64 NumPy oracle of the warm-start network (16 -> 128 -> 128 -> 1,
exact GELU), its mean-squared-error gradient and one Adam step, written from
the textbook definitions (GELU as z * Phi(z) with Phi the normal CDF; Adam with
bias-corrected first and second moments).

TEST INFRASTRUCTURE, like the rest of this package: only the tests may import
it.  Pinned on the CPU by central finite differences of the loss (every
parameter block), the GELU limits and derivative, and the first Adam step.
The trained network's values are parity unpinned: their quality is judged by
the plain qsGW iteration they warm-start."""
import math

import numpy as np

NIN, NHID = 16, 128
SIZES = dict(W1=(NHID, NIN), b1=(NHID,), W2=(NHID, NHID), b2=(NHID,), w3=(NHID,), b3=(1,))
NPARAMS = sum(int(np.prod(s)) for s in SIZES.values())


def unpack(p):
    out, o = {}, 0
    for k, s in SIZES.items():
        n = int(np.prod(s))
        out[k] = np.asarray(p[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for k in SIZES])


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, X):
    q = unpack(p)
    Z1 = X @ q["W1"].T + q["b1"]
    A1 = gelu(Z1)
    Z2 = A1 @ q["W2"].T + q["b2"]
    A2 = gelu(Z2)
    y = A2 @ q["w3"] + q["b3"][0]
    return y, (Z1, A1, Z2, A2)


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64:
    BF16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of
    IEEE binary32, so x is first rounded to binary32, then its low 16 bits
    are rounded off with ties going to the even upper half."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = b & 0xFFFF
    up = b >> 16
    round_up = (low > 0x8000) | ((low == 0x8000) & ((up & 1) == 1))
    up = up + round_up.astype(np.uint64)
    return (up << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, X):
    """The network with BF16 operands: X, W1, the hidden activations, W2 and
    w3 rounded by ``to_bf16``; sums, biases and GELU exact (FP64 here)."""
    q = unpack(p)
    A1 = to_bf16(gelu(to_bf16(X) @ to_bf16(q["W1"]).T + q["b1"]))
    A2 = to_bf16(gelu(A1 @ to_bf16(q["W2"]).T + q["b2"]))
    return A2 @ to_bf16(q["w3"]) + q["b3"][0], (A1, A2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def grad(p, X, t):
    q = unpack(p)
    n = X.shape[0]
    y, (Z1, A1, Z2, A2) = forward(p, X)
    dy = 2.0 * (y - t) / n
    g = {}
    g["w3"] = A2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dZ2 = np.outer(dy, q["w3"]) * gelu_grad(Z2)
    g["W2"] = dZ2.T @ A1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ q["W2"]) * gelu_grad(Z1)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed):
    """Kaiming-uniform-like initialisation."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = rng.uniform(-1, 1, SIZES["W1"]) / math.sqrt(NIN)
    d["b1"] = np.zeros(NHID)
    d["W2"] = rng.uniform(-1, 1, SIZES["W2"]) / math.sqrt(NHID)
    d["b2"] = np.zeros(NHID)
    d["w3"] = rng.uniform(-1, 1, NHID) / math.sqrt(NHID)
    d["b3"] = np.zeros(1)
    return pack(d)
