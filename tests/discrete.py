"""Grid incidence operators for manufactured solutions in the tests.

G (node -> edge gradient) and C (edge -> facet circulation) of the voxel grid,
written with numpy slicing.  They build inputs whose exact discrete answer is
known (a = -G psi* + M^-1 C^T W gives psi = psi* up to a constant and
u = M^-1 C^T W, because C G = 0), and they check Stokes' theorem for the source
generators.  Edge arrays are (3, nz+1, ny+1, nx+1); facet arrays are
(3, nz+1, ny+1, nx+1) with W[d] the facet whose normal is e_d and whose lowest
corner is the node; entries that leave the grid are 0.
"""
import numpy as np


def grad(psi):
    """(G psi)_e = psi(head) - psi(tail) for the edge from node n to n + e_d."""
    Nz, Ny, Nx = psi.shape
    g = np.zeros((3, Nz, Ny, Nx))
    g[0, :, :, :-1] = psi[:, :, 1:] - psi[:, :, :-1]
    g[1, :, :-1, :] = psi[:, 1:, :] - psi[:, :-1, :]
    g[2, :-1, :, :] = psi[1:, :, :] - psi[:-1, :, :]
    return g


def div_T(e):
    """G^T e at the nodes: sum over entering edges minus sum over leaving edges."""
    _, Nz, Ny, Nx = e.shape
    out = np.zeros((Nz, Ny, Nx))
    out[:, :, 1:] += e[0, :, :, :-1]
    out[:, :, :-1] -= e[0, :, :, :-1]
    out[:, 1:, :] += e[1, :, :-1, :]
    out[:, :-1, :] -= e[1, :, :-1, :]
    out[1:, :, :] += e[2, :-1, :, :]
    out[:-1, :, :] -= e[2, :-1, :, :]
    return out


def curl(a):
    """(C a)_f: circulation of the edge field around each facet (right-hand rule)."""
    _, Nz, Ny, Nx = a.shape
    f = np.zeros_like(a)
    ax, ay, az = a
    # normal x, facet spans (j..j+1, k..k+1) at i: y(i,j,k) + z(i,j+1,k) - y(i,j,k+1) - z(i,j,k)
    f[0, :-1, :-1, :] = ay[:-1, :-1, :] + az[:-1, 1:, :] - ay[1:, :-1, :] - az[:-1, :-1, :]
    # normal y, spans (k..k+1, i..i+1) at j: z(i,j,k) + x(i,j,k+1) - z(i+1,j,k) - x(i,j,k)
    f[1, :-1, :, :-1] = az[:-1, :, :-1] + ax[1:, :, :-1] - az[:-1, :, 1:] - ax[:-1, :, :-1]
    # normal z, spans (i..i+1, j..j+1) at k: x(i,j,k) + y(i+1,j,k) - x(i,j+1,k) - y(i,j,k)
    f[2, :, :-1, :-1] = ax[:, :-1, :-1] + ay[:, :-1, 1:] - ax[:, 1:, :-1] - ay[:, :-1, :-1]
    return f


def curl_T(W):
    """C^T W: each facet value is added to its four edges with the orientation sign."""
    _, Nz, Ny, Nx = W.shape
    e = np.zeros_like(W)
    w0 = W[0, :-1, :-1, :]
    e[1, :-1, :-1, :] += w0
    e[2, :-1, 1:, :] += w0
    e[1, 1:, :-1, :] -= w0
    e[2, :-1, :-1, :] -= w0
    w1 = W[1, :-1, :, :-1]
    e[2, :-1, :, :-1] += w1
    e[0, 1:, :, :-1] += w1
    e[2, :-1, :, 1:] -= w1
    e[0, :-1, :, :-1] -= w1
    w2 = W[2, :, :-1, :-1]
    e[0, :, :-1, :-1] += w2
    e[1, :, :-1, 1:] += w2
    e[0, :, 1:, :-1] -= w2
    e[1, :, :-1, :-1] -= w2
    return e


def body_facet_mask(body):
    """Facets that belong to at least one body voxel (all four of their edges conduct)."""
    nz, ny, nx = body.shape
    m = np.zeros((3, nz + 1, ny + 1, nx + 1), bool)
    # voxel (i,j,k) owns facets: normal x at i and i+1 (spanning j,k), etc.
    m[0, :nz, :ny, :nx] |= body
    m[0, :nz, :ny, 1:nx + 1] |= body
    m[1, :nz, :ny, :nx] |= body
    m[1, :nz, 1:ny + 1, :nx] |= body
    m[2, :nz, :ny, :nx] |= body
    m[2, 1:nz + 1, :ny, :nx] |= body
    return m


def manufactured(M, body, rng, psi_scale=1e-6, w_scale=1e-9, smooth=True):
    """Inputs a with a known exact discrete answer.

    psi* = smooth cosines + 1 % noise on all nodes; W random on body facets.
    a = -G psi* + M^-1 C^T W on conducting edges (0 elsewhere).
    Returns (a, psi*, u_exact) with u_exact = M^-1 C^T W (0 on M = 0 edges).
    """
    nz, ny, nx = body.shape
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    psi = np.zeros((nz + 1, ny + 1, nx + 1))
    if smooth:
        psi += np.cos(2 * np.pi * i / max(nx, 1) * 1.3) * np.cos(2 * np.pi * j / max(ny, 1) * 0.7 + 0.3) \
            * np.cos(2 * np.pi * k / max(nz, 1) * 0.9 + 0.1)
    psi += 0.01 * rng.standard_normal(psi.shape)
    psi *= psi_scale
    W = rng.standard_normal((3, nz + 1, ny + 1, nx + 1)) * w_scale
    W *= body_facet_mask(body)
    ctw = curl_T(W)
    cond = M > 0
    u = np.zeros_like(M)
    u[cond] = ctw[cond] / M[cond]
    a = -grad(psi) + u
    a[~cond] = 0.0
    return a, psi, u


def project_mean_zero(x, comp):
    """Subtract the mean over each component (comp = -1 marks non-DOF nodes, set to 0)."""
    out = np.zeros_like(x)
    for c in np.unique(comp[comp >= 0]):
        sel = comp == c
        out[sel] = x[sel] - x[sel].mean()
    return out


def voxel_emag_bruteforce(u, body, h, omega):
    """|E| per voxel by listing each voxel's 12 edges from its 8 corners."""
    nz, ny, nx = body.shape
    E = np.zeros((nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if not body[k, j, i]:
                    continue
                comp = []
                for d in range(3):
                    s = 0.0
                    for c in range(8):
                        ci, cj, ck = c & 1, (c >> 1) & 1, (c >> 2) & 1
                        corner = (ci, cj, ck)
                        if corner[d] != 0:
                            continue          # an edge along d starts at a corner with 0 along d
                        s += u[d, k + ck, j + cj, i + ci]
                    comp.append(s / 4.0 / h[d])
                E[k, j, i] = omega * np.sqrt(sum(x * x for x in comp))
    return E


def project_mean_zero_fast(x, comp, ncomp):
    """project_mean_zero for large grids: per-component means by bincount (comp = -1 marks non-DOF
    nodes, set to 0); the same arithmetic definition, summed in a different order."""
    c = comp.reshape(-1)
    v = x.reshape(-1)
    sel = c >= 0
    sums = np.bincount(c[sel], weights=v[sel], minlength=ncomp)
    cnt = np.bincount(c[sel], minlength=ncomp)
    out = np.zeros_like(v)
    out[sel] = v[sel] - (sums / np.maximum(cnt, 1))[c[sel]]
    return out.reshape(x.shape)
