"""Pins of the learned-preconditioner oracle (features, MLP forward/backward)."""
import numpy as np
import pytest
import torch

from oracle import precond as P
from paper_2602_12365_amd import inputs as I


def rand_theta(seed, scale=0.3):
    return scale * np.random.default_rng(seed).standard_normal(P.N_PARAMS)


def test_bf16_round_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(-5, 5, 10000)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(P.bf16_round(x), ref)


def test_mlp_backward_matches_finite_differences():
    th = rand_theta(1)
    X = np.random.default_rng(2).standard_normal((7, P.N_IN))
    dout = np.random.default_rng(3).standard_normal((7, P.N_OUT))
    g = P.mlp_backward(th, X, dout, rounding=False)
    h = 1e-6
    for k in np.random.default_rng(4).choice(P.N_PARAMS, 40, replace=False):
        e = np.zeros(P.N_PARAMS)
        e[k] = h
        fp = np.sum(dout * P.mlp_forward(th + e, X, rounding=False))
        fm = np.sum(dout * P.mlp_forward(th - e, X, rounding=False))
        assert abs((fp - fm) / (2 * h) - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_mlp_matches_torch_autograd():
    th = rand_theta(5)
    X = np.random.default_rng(6).standard_normal((11, P.N_IN))
    dout = np.random.default_rng(7).standard_normal((11, P.N_OUT))
    t = torch.tensor(th, requires_grad=True)
    parts, k = {}, 0
    for name, shp in P.SHAPES:
        n = int(np.prod(shp))
        parts[name] = t[k:k + n].reshape(shp)
        k += n
    x = torch.tensor(X)
    h1 = torch.nn.functional.softplus(x @ parts["W1"].T + parts["b1"])
    h2 = torch.nn.functional.softplus(h1 @ parts["W2"].T + parts["b2"])
    out = h2 @ parts["W3"].T + parts["b3"]
    (out * torch.tensor(dout)).sum().backward()
    assert np.allclose(out.detach().numpy(), P.mlp_forward(th, X, rounding=False), rtol=1e-13, atol=1e-13)
    assert np.allclose(t.grad.numpy(), P.mlp_backward(th, X, dout, rounding=False), rtol=1e-12, atol=1e-12)


def test_mlp_layers_compose_to_the_forward_pass():
    """The per-layer form used for layer-by-layer parity is the rounded
    forward pass, layer by layer, to the last bit."""
    th = rand_theta(8)
    X = P.bf16_round(np.random.default_rng(9).standard_normal((33, P.N_IN)).astype(np.float32))
    out, (x0, a1, h1, a2, h2, p) = P.mlp_forward(th, X, keep=True)
    assert np.array_equal(P.mlp_layer(th, 1, x0), h1)
    assert np.array_equal(P.mlp_layer(th, 2, h1), h2)
    assert np.array_equal(P.mlp_layer(th, 3, h2), out)
    assert np.all(P.mlp_layer(th, 1, x0) > 0)


def brute_features(r, D, M, conn, n):
    nb = [set() for _ in range(n)]
    for ce in conn:
        for a in ce:
            for b in ce:
                if a != b:
                    nb[a].add(int(b))
    F = np.zeros((n, 12))
    s_all = np.zeros(n)
    g = np.zeros((n, 3))
    for i in range(n):
        for c in range(3):
            g[i, c] = 0.0 if M[i, c] else r[i, c] / D[i, c]
    for i in range(n):
        js = sorted(nb[i])
        s = np.sqrt((np.sum(g[i] ** 2) + sum(np.sum(g[j] ** 2) for j in js)) / (3 * (len(js) + 1)))
        s_all[i] = s
        if s > 0:
            F[i, 0:3] = g[i] / s
            F[i, 3:6] = sum(g[j] for j in js) / len(js) / s
        for c in range(3):
            F[i, 6 + c] = np.log(D[i, c] / ((D[i, c] + sum(D[j, c] for j in js)) / (len(js) + 1)))
        F[i, 9] = M[i].sum() / 3
        F[i, 10] = sum(M[j].sum() for j in js) / (3 * len(js))
        F[i, 11] = len(js) / 26
    return F, s_all


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_features_match_brute_force(elem):
    m = I.make_mesh(elem, 2)
    rng = np.random.default_rng(8)
    r = rng.standard_normal((m.n_nodes, 3))
    D = rng.uniform(0.5, 2.0, (m.n_nodes, 3))
    mask, _ = I.clamp_top_bottom(m.X, 0.1, top_all_components=False)
    M = mask.reshape(-1, 3) != 0
    ptr, idx = P.node_neighbours(m.conn, m.n_nodes)
    F, g, s = P.features(r, D, mask, ptr, idx)
    Fb, sb = brute_features(r, D, M, m.conn, m.n_nodes)
    assert np.allclose(F, Fb, rtol=1e-12, atol=1e-12)
    assert np.allclose(s, sb, rtol=1e-12, atol=0)
    if elem == I.HEX8:
        assert np.diff(ptr).max() == 26       # interior node of a hex grid


def test_apply_is_positively_homogeneous_and_masked():
    m = I.hex_mesh(3)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((m.n_nodes, 3))
    D = rng.uniform(0.5, 2.0, (m.n_nodes, 3))
    mask, _ = I.clamp_top_bottom(m.X, 0.1)
    ptr, idx = P.node_neighbours(m.conn, m.n_nodes)
    th = rand_theta(10)
    z = P.apply(th, r, D, mask, ptr, idx)
    assert np.array_equal(P.apply(th, 4.0 * r, D, mask, ptr, idx), 4.0 * z)
    assert np.all(z.reshape(-1)[mask != 0] == 0)
    # the zero network is Jacobi
    zj = P.apply(np.zeros(P.N_PARAMS), r, D, mask, ptr, idx)
    assert np.allclose(zj, np.where(mask.reshape(-1, 3) != 0, 0, r / D))


def test_apply_safeguard_keeps_half_the_jacobi_share_per_node():
    """r_i . z_i >= r_i . g_i / 2 at every node, with equality exactly where the
    correction was scaled back; elsewhere z = g + s MLP unchanged."""
    m = I.hex_mesh(3)
    rng = np.random.default_rng(11)
    r = rng.standard_normal((m.n_nodes, 3))
    D = rng.uniform(0.5, 2.0, (m.n_nodes, 3))
    mask, _ = I.clamp_top_bottom(m.X, 0.1)
    ptr, idx = P.node_neighbours(m.conn, m.n_nodes)
    th = rand_theta(12, 1.0)                    # large weights: many nodes need the safeguard
    z = P.apply(th, r, D, mask, ptr, idx)
    F, g, s = P.features(r, D, mask, ptr, idx)
    c = s[:, None] * P.mlp_forward(th, F.astype(np.float32))
    c[mask.reshape(-1, 3) != 0] = 0.0
    a = (r * g).sum(axis=1)
    rz = (r * z).sum(axis=1)
    low = a + (r * c).sum(axis=1) < 0.5 * a
    assert low.sum() > 5 and (~low).sum() > 5
    assert np.all(rz >= 0.5 * a - 1e-12 * np.abs(a).max())
    assert np.allclose(rz[low], 0.5 * a[low], rtol=1e-12, atol=1e-14)
    assert np.allclose(z[~low], (g + c)[~low], rtol=0, atol=0)
    assert (r * z).sum() >= 0.5 * (r * g).sum()
