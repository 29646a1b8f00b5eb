"""FP64 oracle of the learned CG preconditioner: node features, the per-node
MLP (forward and backward) and the preconditioner apply.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper uses small softplus MLPs as energy terms (Sec. 6.6.1, Eq. 17); the
preconditioner built here is this project's own addition, so nothing in it is
pinned by the paper: its definition is the reading below, and its pins are
mathematical (finite differences of the MLP loss, an independent autograd,
brute-force feature loops on tiny meshes, homogeneity of the apply).

Definition (per node i, with N(i) the nodes sharing an element with i):
    g_i   = D_i^-1 r_i  (Jacobi-scaled residual, 0 on prescribed DOFs)
    s_i   = sqrt( (|g_i|^2 + sum_{j in N(i)} |g_j|^2) / (3 (|N(i)| + 1)) )
    f_i   = [ g_i / s_i,                                  (3)
              mean_{j in N(i)} g_j / s_i,                 (3)
              log(D_ic / mean_{j in N(i) + i} D_jc), c=0..2  (3)
              prescribed fraction of node i's 3 DOFs,     (1)
              prescribed fraction of the DOFs of N(i),    (1)
              |N(i)| / 26 ]                               (1)
    z_i   = g_i + s_i * MLP(f_i), prescribed DOFs -> 0
MLP: 12 -> 64 -> 64 -> 3, softplus on the hidden layers; weights and layer
inputs rounded to bfloat16 (round to nearest even), arithmetic in FP64 here.
Nodes with s_i = 0 get z_i = g_i (= 0).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 12, 64, 3
# flat parameter layout: W1 [64,12], b1 [64], W2 [64,64], b2 [64], W3 [3,64], b3 [3]
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def mlp_forward(theta, X, keep=False, rounding=True):
    """X [n, 12] -> out [n, 3]; weights and every layer input rounded to bf16
    (rounding=False: the same network in plain FP64, for derivative pins)."""
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    p = {k: rnd(v) for k, v in unpack(theta).items()}
    x0 = rnd(X)
    a1 = x0 @ p["W1"].T + p["b1"]
    h1 = rnd(softplus(a1))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = rnd(softplus(a2))
    out = h2 @ p["W3"].T + p["b3"]
    if keep:
        return out, (x0, a1, h1, a2, h2, p)
    return out


def mlp_layer(theta, k, inp):
    """One layer of mlp_forward (rounded form) applied to a given layer
    input: k = 1, 2 the hidden layers, bf16(softplus(W_k inp + b_k)) with inp
    [n, 12] or [n, 64]; k = 3 the output W3 inp + b3.  The input is used as
    given (bf16 values already), so a test can evaluate each layer on another
    implementation's own rounded activations."""
    p = {name: bf16_round(v) for name, v in unpack(theta).items()}
    a = np.asarray(inp, dtype=np.float64) @ p[f"W{k}"].T + p[f"b{k}"]
    return a if k == 3 else bf16_round(softplus(a))


def mlp_backward(theta, X, dout, rounding=True):
    """Gradient of sum(dout * out) with respect to the flat parameters (the
    bf16 roundings are treated as identity, as in a straight-through estimate)."""
    _, (x0, a1, h1, a2, h2, p) = mlp_forward(theta, X, keep=True, rounding=rounding)
    g = {}
    g["W3"] = dout.T @ h2
    g["b3"] = dout.sum(axis=0)
    dh2 = dout @ p["W3"]
    dz2 = dh2 * sigmoid(a2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * sigmoid(a1)
    g["W1"] = dz1.T @ x0
    g["b1"] = dz1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def node_neighbours(conn, n_nodes):
    """CSR (ptr, idx) of N(i): nodes sharing an element with i, excluding i, sorted."""
    conn = np.asarray(conn, dtype=np.int64)
    nen = conn.shape[1]
    a = np.repeat(conn, nen, axis=1).ravel()
    b = np.tile(conn, (1, nen)).ravel()
    keep = a != b
    pairs = np.unique(np.stack([a[keep], b[keep]], axis=1), axis=0)
    ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(ptr, pairs[:, 0] + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, pairs[:, 1]


def features(r, diag, mask, ptr, idx):
    """Node features and scales: returns (F [n, 12], g [n, 3], s [n])."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    D = np.asarray(diag, dtype=np.float64).reshape(-1, 3)
    M = np.asarray(mask).reshape(-1, 3) != 0
    n = r.shape[0]
    g = np.where(M, 0.0, r / D)
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(n), deg)
    sum_g = np.zeros((n, 3))
    np.add.at(sum_g, rows, g[idx])
    sum_g2 = np.zeros(n)
    np.add.at(sum_g2, rows, (g[idx] ** 2).sum(axis=1))
    sum_D = np.zeros((n, 3))
    np.add.at(sum_D, rows, D[idx])
    sum_M = np.zeros(n)
    np.add.at(sum_M, rows, M[idx].sum(axis=1))
    s = np.sqrt(((g ** 2).sum(axis=1) + sum_g2) / (3.0 * (deg + 1)))
    safe = np.where(s > 0, s, 1.0)
    F = np.zeros((n, N_IN))
    F[:, 0:3] = g / safe[:, None]
    F[:, 3:6] = sum_g / np.maximum(deg, 1)[:, None] / safe[:, None]
    F[:, 6:9] = np.log(D / ((sum_D + D) / (deg + 1)[:, None]))
    F[:, 9] = M.sum(axis=1) / 3.0
    F[:, 10] = sum_M / (3.0 * np.maximum(deg, 1))
    F[:, 11] = deg / 26.0
    F[s == 0, 0:6] = 0.0
    return F, g, s


def apply(theta, r, diag, mask, ptr, idx):
    """z = g + gamma * s * MLP(features), prescribed DOFs 0, with the node-wise
    safeguard gamma in (0, 1]: where the correction c = s * MLP would leave
    r_i . z_i below half of r_i . g_i (the Jacobi step's share), it is scaled
    back to exactly half, so that r . z >= r . D^-1 r / 2 > 0 for r != 0."""
    F, g, s = features(r, diag, mask, ptr, idx)
    out = mlp_forward(theta, F.astype(np.float32))
    fixed = np.asarray(mask).reshape(-1, 3) != 0
    c = s[:, None] * out
    c[s == 0] = 0.0
    c[fixed] = 0.0
    R = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    a = (R * g).sum(axis=1)
    b = (R * c).sum(axis=1)
    low = a + b < 0.5 * a
    gamma = np.ones_like(a)
    gamma[low] = -0.5 * a[low] / b[low]
    return g + gamma[:, None] * c
