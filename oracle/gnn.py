"""Float64 reference of the learned proposal's network -- TEST INFRASTRUCTURE.

Forward and hand-written backward of the message-passing network used to
score variables for slicing and for elimination (see the library header for
the architecture): three layers H' = relu(H Ws + mean_{w in N(v)} H[w] Wn + b)
of width 64 over 8 input features shared by two linear heads s_h = H w_h +
c_h (0: slicing, 1: elimination), and the loss mean_i (s_h[cand_i] - y_i)^2.
Parameters are the flat vector of the library (layer by layer Ws[din][64],
Wn[din][64], b[64]; then head 0 (w[64], c), then head 1 (w[64], c)).  The
backward pass is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

F, H, L = 8, 64, 3
HEADS = 2


def unpack(p, head=0):
    p = np.asarray(p, dtype=np.float64)
    layers = []
    o = 0
    for l in range(L):
        din = F if l == 0 else H
        ws = p[o:o + din * H].reshape(din, H); o += din * H
        wn = p[o:o + din * H].reshape(din, H); o += din * H
        b = p[o:o + H]; o += H
        layers.append((ws, wn, b))
    o += head * (H + 1)
    w = p[o:o + H]; o += H
    c = p[o]
    return layers, w, c


def n_params():
    return sum(2 * (F if l == 0 else H) * H + H for l in range(L)) + HEADS * (H + 1)


def mean_agg(A, X):
    """A: dense 0/1 symmetric adjacency (n x n); mean over neighbours."""
    deg = A.sum(axis=1)
    M = A @ X
    nz = deg > 0
    M[nz] /= deg[nz, None]
    M[~nz] = 0.0
    return M


def forward(p, A, X, head=0):
    layers, w, c = unpack(p, head)
    Hs, Ms, Zs = [np.asarray(X, dtype=np.float64)], [], []
    for ws, wn, b in layers:
        M = mean_agg(A, Hs[-1])
        Z = Hs[-1] @ ws + M @ wn + b
        Ms.append(M)
        Zs.append(Z)
        Hs.append(np.maximum(Z, 0.0))
    s = Hs[-1] @ w + c
    return s, (Hs, Ms, Zs)


def loss_and_grad(p, A, X, cand, y, head=0):
    layers, w, c = unpack(p, head)
    s, (Hs, Ms, Zs) = forward(p, A, X, head)
    cand = np.asarray(cand)
    d = s[cand] - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(d ** 2))
    dS = np.zeros_like(s)
    dS[cand] = 2.0 * d / len(cand)
    grads = []
    gw = Hs[-1].T @ dS
    gc = dS.sum()
    dH = np.outer(dS, w)
    deg = A.sum(axis=1)
    inv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)
    for l in range(L - 1, -1, -1):
        ws, wn, b = layers[l]
        dZ = dH * (Zs[l] > 0)
        gws = Hs[l].T @ dZ
        gwn = Ms[l].T @ dZ
        gb = dZ.sum(axis=0)
        grads.append((gws, gwn, gb))
        dHs = dZ @ ws.T
        dM = dZ @ wn.T
        dH = dHs + A.T @ (dM * inv[:, None])
    grads.reverse()
    flat = []
    for gws, gwn, gb in grads:
        flat += [gws.ravel(), gwn.ravel(), gb]
    for h in range(HEADS):  # the loss reaches only the scored head
        flat += [gw, np.array([gc])] if h == head else [np.zeros(H), np.zeros(1)]
    return loss, np.concatenate(flat)
