"""ORACLE — test infrastructure, not product code.

A second, independent, pure-Python walker for tiny sample sizes.  It uses an
explicit stack instead of recursion and Python integers for Philox4x32-10, so a
mistake in ``walker.c`` (recursion order, counter layout, word assignment,
clock rule, weights) shows up as a tree-by-tree disagreement.  It reads the
same normalised problem as ``oracle.normalize`` but none of its code.
"""
from __future__ import annotations

import math

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 on Python ints (Salmon et al., SC'11)."""
    c = [v & _MASK for v in ctr]
    k0, k1 = key[0] & _MASK, key[1] & _MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c[3] ^ k1) & _MASK, p0 & _MASK]
    return c


def _g(kind, p, nterms, dim, x):
    if kind == 0:
        return p[0]
    if kind == 1:
        nx = x[0] * p[4] + (x[1] * p[5] if dim == 2 else 0.0)
        base = 1.0 / (1.0 + math.exp(p[1] * (nx - p[2])))
        return p[0] * base ** int(p[3])
    if kind == 2:
        tot = 0.0
        for k in range(nterms):
            A, cx, cy, s = p[4 * k: 4 * k + 4]
            r2 = (x[0] - cx) ** 2 + ((x[1] - cy) ** 2 if dim == 2 else 0.0)
            tot += A * math.exp(-r2 / (2 * s * s))
        return tot
    if kind == 3:
        if abs(x[0]) > p[1] or (dim == 2 and abs(x[1]) > p[2]):
            return 0.0
        v = p[0] * math.cos(math.pi * x[0] / (2 * p[1])) ** 2
        if dim == 2:
            v *= math.cos(math.pi * x[1] / (2 * p[2])) ** 2
        return v
    raise ValueError(kind)


def _move(nz, key, node, tree, point_id, x, dt, z):
    """End of an edge of duration dt from x (z: the normals of the node's own block): one exact Gaussian
    increment for constant coefficients, else ceil(dt/h) equal Euler-Maruyama steps whose k-th step
    (k >= 1) draws its normals from the Philox block (node, tree, point, k)."""
    dim = nz.dim
    if not nz.euler:
        return [x[d] + nz.drift[d] * dt + nz.sigma * math.sqrt(dt) * z[d] for d in range(dim)]
    bx, by, amp, sk, inv_h = nz.euler
    blin = (bx, by)
    n = min(max(1, int(math.ceil(dt * inv_h))), 1 << 20)  # at most 2^20 steps per edge
    h = dt / n
    sh = math.sqrt(h)
    y = list(x[:dim])
    zz = list(z)
    for k in range(n):
        if k > 0:
            w = philox4x32_10((node, tree, point_id, k), key)
            u1 = (w[2] + 0.5) / 2.0 ** 32
            u2 = w[3] / 2.0 ** 32
            r = math.sqrt(-2.0 * math.log(u1))
            zz = [r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)]
        r2 = sum(y[d] * y[d] for d in range(dim))
        sg = nz.sigma * (1.0 + amp * math.exp(-sk * r2))
        inc = [(nz.drift[d] + blin[d] * y[d]) * h + sg * sh * zz[d] for d in range(dim)]
        y = [y[d] + inc[d] for d in range(dim)]
    return y


def _cmod(nz, x, tau):
    """Scale of the constant coefficients at a split at x with PDE time tau left (variable c_j(x, t))."""
    cm = getattr(nz, "cmod", None)
    if not cm:
        return 1.0
    bx, by, t0, pw = cm
    e = bx * x[0] * x[0] + (by * x[1] * x[1] if len(x) > 1 else 0.0)
    v = math.exp(-e)
    return v / (tau + t0) if pw == 1 else v


def walk_tree(nz, mc, x0, t, point_id, tree):
    """One tree with an explicit stack.  Returns (F, ne, nodes, flags).

    The stack holds, per vertex that still has children to start, the state
    its children depart from (position, clock product, time left) and the
    number of children not yet started.  Every node multiplies its factor
    (vertex weight or g at the leaf) into a running product.
    """
    if getattr(nz, "strategy", 0) == 1:
        return _walk_tree_b(nz, mc, x0, t, point_id, tree)
    seed = int(mc.get("seed", 0))
    key = (seed & _MASK, (seed >> 32) & _MASK)
    K = len(nz.J)
    theta = math.exp(-nz.lam * t) if K > 0 else 1.0
    cap = int(mc.get("node_cap", 1 << 16))
    max_order = int(mc.get("max_order", 12))
    prune = int(mc.get("prune", 1))
    dim = nz.dim
    state = (list(x0[:dim]), 1.0, t)   # departure state of the next node
    stack = []                          # [state, children left]
    node = ne = 0
    prod = 1.0
    while True:
        if node >= cap:
            return 0.0, ne, node, 2
        w = philox4x32_10((node, tree, point_id, 0), key)
        node += 1
        x, P, tau = state
        U = (w[0] + 0.5) / 2.0 ** 32
        Pn = P * U
        u1 = (w[2] + 0.5) / 2.0 ** 32
        u2 = w[3] / 2.0 ** 32
        r = math.sqrt(-2.0 * math.log(u1))
        z = (r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2))
        branch_done = False
        if Pn > theta:
            S = -math.log(U) / nz.lam
            tau2 = max(tau - S, 0.0)
            xs = _move(nz, key, node - 1, tree, point_id, x, S, z)
            ne += 1
            if prune and ne > max_order:
                return 0.0, ne, node, 1
            idx = (w[1] * K) >> 32
            alpha = nz.J[idx]
            prod *= nz.omega[idx] * math.exp((alpha - 1) * nz.mu * tau2) * _cmod(nz, xs, tau2)
            if alpha == 0:
                branch_done = True
            else:
                if alpha > 1:
                    stack.append([(xs, Pn, tau2), alpha - 1])
                state = (xs, Pn, tau2)
        else:
            xl = _move(nz, key, node - 1, tree, point_id, x, tau, z)
            prod *= _g(nz.u0_kind, nz.u0_params, nz.u0_nterms, dim, xl)
            branch_done = True
        if branch_done:
            if not stack:
                return prod, ne, node, 0
            top = stack[-1]
            state = top[0]
            top[1] -= 1
            if top[1] == 0:
                stack.pop()


def _walk_tree_b(nz, mc, x0, t, point_id, tree):
    """Strategy B (coin with P(leaf) = q, split after a uniform fraction of the time left), explicit stack."""
    seed = int(mc.get("seed", 0))
    key = (seed & _MASK, (seed >> 32) & _MASK)
    K = len(nz.J)
    Q = int(math.floor(nz.q * 2.0 ** 32))
    cap = int(mc.get("node_cap", 1 << 16))
    max_order = int(mc.get("max_order", 12))
    prune = int(mc.get("prune", 1))
    dim = nz.dim
    state = (list(x0[:dim]), t)     # departure state of the next node: position, time left
    stack = []
    node = ne = 0
    prod = 1.0
    while True:
        if node >= cap:
            return 0.0, ne, node, 2
        w = philox4x32_10((node, tree, point_id, 0), key)
        node += 1
        x, tau = state
        u1 = (w[2] + 0.5) / 2.0 ** 32
        u2 = w[3] / 2.0 ** 32
        r = math.sqrt(-2.0 * math.log(u1))
        z = (r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2))
        if w[0] >= Q:
            span = 2.0 ** 32 - Q
            s = tau * ((w[0] - Q + 0.5) / span)
            tau2 = tau * ((2 ** 32 - 1 - w[0] + 0.5) / span)  # tau (1 - V) without cancellation
            xs = _move(nz, key, node - 1, tree, point_id, x, s, z)
            ne += 1
            if prune and ne > max_order:
                return 0.0, ne, node, 1
            idx = (w[1] * K) >> 32
            alpha = nz.J[idx]
            prod *= tau * nz.omega[idx] * math.exp((alpha - 1) * nz.mu * tau2) * _cmod(nz, xs, tau2)
            if alpha > 0:
                if alpha > 1:
                    stack.append([(xs, tau2), alpha - 1])
                state = (xs, tau2)
                continue
        else:
            xl = _move(nz, key, node - 1, tree, point_id, x, tau, z)
            prod *= _g(nz.u0_kind, nz.u0_params, nz.u0_nterms, dim, xl) / nz.q
        if not stack:
            return prod, ne, node, 0
        top = stack[-1]
        state = top[0]
        top[1] -= 1
        if top[1] == 0:
            stack.pop()
