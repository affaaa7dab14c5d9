"""TEST INFRASTRUCTURE ONLY: oracle of the learned warm start's grid transfers and of the
optimiser that trains it (only tests, the smoke check and the benchmark's CPU-baseline leg
use it; the GPU library never loads it and shares no code with it).

The paper has no learned part; these are the definitions the library implements for it,
written out plainly in FP64 numpy so that each can be checked by eye:

* Network input of one problem on a grid with n = 4 nc interior points per direction
  (nodes 0 and n + 1 are the walls).  Coarse cell c (per direction) is the block of interior
  nodes 1 + 4c ... 4 + 4c; its value is the mean over the 4^3 nodes of the block.
  sigma = sqrt(mean over ALL nodes of g^2 + (f / 3 pi^2)^2) (1 if that is 0).  Channels:
  0: mean(f) / (3 pi^2 sigma), 1: clamp(mean(phi) nc / 8, -1, 1), 2: mean(g) / sigma.
  Target: mean(v) / sigma with v = u where phi > 0 and v = g where phi <= 0 (the solution
  continued into the bodies by g, which is smooth across the interface where the solution
  jumps to 0).  Arrays are [z][y][x], x fastest, like the node arrays.
* Prolongation of a coarse field p (one value per cell) to the fine nodes, in index space:
  along each axis, fine node i sits at coarse coordinate s = (i - 2.5) / 4 (cell c's centre
  is at fine index 2.5 + 4c), clamped to [0, nc - 1]; the value is the tensor product of
  1D linear (hat-function) interpolation between the two cell centres around s, times
  sigma.  Beyond the outermost cell centres the value is constant.
* Adam (Kingma & Ba, "Adam: A method for stochastic optimization", ICLR 2015, Algorithm 1):
  m_t = b1 m_{t-1} + (1 - b1) g_t, v_t = b2 v_{t-1} + (1 - b2) g_t^2, with bias corrections
  m^_t = m_t / (1 - b1^t), v^_t = v_t / (1 - b2^t), and w_t = w_{t-1} - lr m^_t / (sqrt(v^_t) + eps),
  from m_0 = v_0 = 0.
"""
import numpy as np

THREE_PI2 = 3.0 * np.pi ** 2


def scale_sigma(f, g):
    """sigma = RMS over all nodes of sqrt(g^2 + (f / 3 pi^2)^2); 1 when that is 0."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    s = np.sqrt(np.mean(g * g + (f / THREE_PI2) ** 2))
    return s if s > 0.0 else 1.0


def block_means(a, nc):
    """Means over the 4^3 blocks of interior nodes: a is a node array [(4nc+2)]^3, the
    result [nc]^3 with cell (cz, cy, cx) = mean of a[1+4cz:5+4cz, 1+4cy:5+4cy, 1+4cx:5+4cx]."""
    a = np.asarray(a, dtype=np.float64)
    assert a.shape == (4 * nc + 2,) * 3, (a.shape, nc)
    inner = a[1:-1, 1:-1, 1:-1]
    return inner.reshape(nc, 4, nc, 4, nc, 4).mean(axis=(1, 3, 5))


def restrict_inputs(f, phi, g, nc):
    """Network input [3][nc]^3 of one problem and its sigma."""
    sigma = scale_sigma(f, g)
    out = np.empty((3, nc, nc, nc))
    out[0] = block_means(f, nc) / (THREE_PI2 * sigma)
    out[1] = np.clip(block_means(phi, nc) * nc / 8.0, -1.0, 1.0)
    out[2] = block_means(g, nc) / sigma
    return out, sigma


def restrict_target(u, phi, g, sigma, nc):
    """Training target [nc]^3: the cell means of (u where phi > 0, else g) / sigma."""
    v = np.where(np.asarray(phi) > 0.0, np.asarray(u, dtype=np.float64), np.asarray(g, dtype=np.float64))
    return block_means(v, nc) / sigma


def hat_matrix(n_fine, nc):
    """1D prolongation in index space: P[i, c] is the weight of cell c at fine node i."""
    P = np.zeros((n_fine, nc))
    for i in range(n_fine):
        s = min(max((i - 2.5) / 4.0, 0.0), nc - 1.0)
        for c in range(nc):
            P[i, c] = max(0.0, 1.0 - abs(s - c))
    return P


def prolong(p, sigma, shape):
    """u0 on the fine nodes (shape = (nz, ny, nx)) from the coarse field p [nc]^3."""
    p = np.asarray(p, dtype=np.float64)
    nc = p.shape[0]
    Pz, Py, Px = (hat_matrix(n, nc) for n in shape)
    return sigma * np.einsum("kc,jb,ia,cba->kji", Pz, Py, Px, p)


def adam(w0, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Parameters after one Adam step per gradient in `grads` (a list), from zero moments."""
    w = np.array(w0, dtype=np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    out = []
    for t, g in enumerate(grads, start=1):
        g = np.asarray(g, dtype=np.float64)
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * g * g
        mhat = m / (1.0 - b1 ** t)
        vhat = v / (1.0 - b2 ** t)
        w = w - lr * mhat / (np.sqrt(vhat) + eps)
        out.append(w.copy())
    return out
