"""Oracle values at single nodes of a large one-plane grid, from a window
around each node (test helper).

After m RK4 steps a node depends only on nodes at most 4 m cells away per axis:
the stencil input of stage s is formed from Y and G_{s-2} at most (phi_t =
psi), so a step reaches 2 + 2 cells.  A window that extends R >= 4 m cells
beyond the node on every side (or to the grid's edge, where its zero halo is
the grid's own) therefore gives the node the same value as the whole grid;
the per-node arithmetic does not depend on the grid size, so the value is
bitwise the same.  The default R = 4 m + 8 leaves a margin."""
import numpy as np


def window_solve(oracle, phi0, y, x, w, steps, R=None):
    R = 4 * steps + 8 if R is None else R
    ny, nx = phi0.shape[1:]
    y0, y1 = max(0, y - R), min(ny, y + R + 1)
    x0, x1 = max(0, x - R), min(nx, x + R + 1)
    win = np.ascontiguousarray(phi0[:, y0:y1, x0:x1])
    p, s = oracle.solve(win, np.zeros_like(win), w.h, w.mu2, w.lam, w.dt, steps, t0=w.t0,
                        inv_L2=w.inv_L2)
    return p[0, y - y0, x - x0], s[0, y - y0, x - x0]


def sample_nodes(ny, nx, seed=11, count=6):
    """Corners, edge midpoints, nodes next to the edges, the centre and seeded
    random nodes (y, x)."""
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (ny - 1, nx // 2), (ny // 2, nx - 1),
           (1, 2), (ny - 2, nx - 3), (ny // 2, nx // 2)]
    rng = np.random.default_rng(seed)
    pts += [(int(rng.integers(ny)), int(rng.integers(nx))) for _ in range(count)]
    return pts


def window_solve3(oracle, phi0, phi1, z, y, x, w, steps, R=None):
    """As window_solve, on a window in all three axes around node (z, y, x)
    of a 3-D grid with initial data (phi0, phi1).  Returns the node's
    (phi, psi) and the window's largest |phi|, |psi| after the steps."""
    R = 4 * steps + 8 if R is None else R
    nz, ny, nx = phi0.shape
    z0, z1 = max(0, z - R), min(nz, z + R + 1)
    y0, y1 = max(0, y - R), min(ny, y + R + 1)
    x0, x1 = max(0, x - R), min(nx, x + R + 1)
    p0 = np.ascontiguousarray(phi0[z0:z1, y0:y1, x0:x1])
    p1 = np.ascontiguousarray(phi1[z0:z1, y0:y1, x0:x1])
    p, s = oracle.solve(p0, p1, w.h, w.mu2, w.lam, w.dt, steps, t0=w.t0, inv_L2=w.inv_L2)
    return (p[z - z0, y - y0, x - x0], s[z - z0, y - y0, x - x0],
            max(float(np.max(np.abs(p))), float(np.max(np.abs(s)))))
