"""FP64 reference of the learned start: a small MLP on occupation strings.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Nothing of the method in
the paper is learned; this network only proposes a Lanczos start vector, so
its definition is this project's reading (documented with the design):

* input: 32 features, x_i = 2 n_i - 1 for the up occupation of site i
  (i < 16) and x_{16+i} = 2 n_i - 1 for the down occupation of site i;
* two hidden layers of 128 units with tanh, one linear output layer of 2:
  o_0 is the log-amplitude ln|psi|, o_1 the logit of P(sign psi > 0);
* parameters in one vector, in this order: W1 (128 x 32, row = unit),
  b1 (128), W2 (128 x 128), b2 (128), W3 (2 x 128), b3 (2): 20,994 values;
* loss over a minibatch of n states drawn with probability ~ |psi|^2:
  (1/n) sum [(o_0 - ln|psi|)^2 + softplus(o_1) - y o_1], y = 1 if psi > 0;
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) on FP32 master weights.

The device kernels compute in BF16 (weights, features, stored activations)
with FP32 accumulation.  `round_bf16=True` rounds the same quantities here
(round to nearest even) so that the two can be compared closely; all other
arithmetic is FP64.  The backward pass treats the rounding as the identity,
as the device does.
"""
import numpy as np

N_IN, N_HID, N_OUT = 32, 128, 2
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    """Views of the parameter vector as the named arrays."""
    out, k = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape)
        k += n
    return out


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), computed from the FP32 value."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(up, dn):
    """32 features per state from up and down occupation strings (sites 0..15)."""
    up = np.asarray(up, dtype=np.uint64)
    dn = np.asarray(dn, dtype=np.uint64)
    x = np.empty((len(up), N_IN), dtype=np.float64)
    for i in range(16):
        x[:, i] = 2.0 * ((up >> np.uint64(i)) & np.uint64(1)).astype(np.float64) - 1.0
        x[:, 16 + i] = 2.0 * ((dn >> np.uint64(i)) & np.uint64(1)).astype(np.float64) - 1.0
    return x


def forward(theta, up, dn, round_bf16=True):
    """Outputs (n x 2) and the cache for backward."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    r = bf16_round if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (r(p[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    x = features(up, dn)
    h1 = r(np.tanh(x @ W1.T + b1))
    h2 = r(np.tanh(h1 @ W2.T + b2))
    out = h2 @ W3.T + b3
    return out, {"x": x, "h1": h1, "h2": h2, "W2": W2, "W3": W3}


def loss_and_dout(out, logamp, sign):
    """Mean loss and its gradient with respect to the outputs."""
    n = out.shape[0]
    a, s = out[:, 0], out[:, 1]
    y = (np.asarray(sign) > 0).astype(np.float64)
    softplus = np.logaddexp(0.0, s)
    loss = float(np.sum((a - logamp) ** 2 + softplus - y * s) / n)
    dout = np.empty_like(out)
    dout[:, 0] = 2.0 * (a - logamp) / n
    dout[:, 1] = (1.0 / (1.0 + np.exp(-s)) - y) / n
    return loss, dout


def backward(cache, dout):
    """Gradient of sum(dout * out) with respect to the parameter vector (chain rule by hand)."""
    x, h1, h2, W2, W3 = cache["x"], cache["h1"], cache["h2"], cache["W2"], cache["W3"]
    g = {}
    g["W3"] = dout.T @ h2
    g["b3"] = dout.sum(axis=0)
    dz2 = (dout @ W3) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed):
    """Uniform fan-in initialisation: each weight in +-1/sqrt(fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(N_PARAMS)
    p = unpack(theta)
    for name, fan in (("W1", N_IN), ("W2", N_HID), ("W3", N_HID)):
        p[name][...] = rng.uniform(-1.0, 1.0, p[name].shape) / np.sqrt(fan)
    return theta


# ---------------------------------------------------------------- sampling

def quantised_weights(psi):
    """Integer sampling weights w_r = floor(2^32 psi_r^2 / max psi^2): exact in any summation order."""
    p2 = np.asarray(psi, dtype=np.float64) ** 2
    m = p2.max()
    return np.floor(p2 / m * 4294967296.0).astype(np.uint64)


def sample_indices(psi, seed, first, count):
    """Indices drawn with probability w_r / sum w: for draw j, the SplitMix64 output
    number first + j of `seed` is scaled to t = floor(z * W / 2^64) and the index is
    the first r whose inclusive prefix sum of w exceeds t."""
    from .splitmix import splitmix64_mix, GAMMA, MASK
    prefix = np.cumsum(quantised_weights(psi), dtype=np.uint64)
    W = int(prefix[-1])
    out = np.empty(count, dtype=np.int64)
    for j in range(count):
        z = splitmix64_mix((seed + (first + j + 1) * GAMMA) & MASK)
        t = (z * W) >> 64
        out[j] = int(np.searchsorted(prefix, np.uint64(t), side="right"))
    return out


def start_vector(theta, up_list, dn_list, round_bf16=True):
    """Unnormalised learned start vector over the whole basis, r = i_up * D_dn + i_dn:
    v_r = (+1 if o_1 >= 0 else -1) * exp(min(o_0, 60))."""
    up = np.repeat(np.asarray(up_list, dtype=np.uint64), len(dn_list))
    dn = np.tile(np.asarray(dn_list, dtype=np.uint64), len(up_list))
    out, _ = forward(theta, up, dn, round_bf16=round_bf16)
    return np.where(out[:, 1] >= 0.0, 1.0, -1.0) * np.exp(np.minimum(out[:, 0], 60.0))
