"""Structured triangle-split mesh, Taylor-Hood P2-P1 DoF maps and Vanka+star
patches (oracle).

Mesh (Sec. 4): the unit square cut into M x M squares, each split along the
diagonal from bottom-right to top-left.  Vertex v = i + (M+1) j sits at
(i/M, j/M).  Square (i, j) gives the cells (v_ij, v_i+1,j, v_i,j+1) and
(v_i+1,j+1, v_i,j+1, v_i+1,j).  P2 nodes (vertices and edge midpoints) form
the (2M+1)^2 grid of spacing h/2; node g = gi + (2M+1) gj.

Free-DoF numbering (the layout every space-time vector uses): interior P2 node
k = (gi-1) + (2M-1)(gj-1) owns velocity DoFs 2k (x) and 2k+1 (y); pressure at
vertex v is DoF 2 (2M-1)^2 + v.  Dirichlet velocity DoFs on the boundary are
not unknowns.  A space-time vector is indexed [free DoF][slab n][temporal node a].

Patches (Sec. 3, Vanka+star, Fig. patches): one per vertex, including boundary
vertices; it holds every free velocity DoF of every P2 node in the closure of
the vertex star (all nodes of the incident cells) and the pressure DoF at the
vertex (the only P1 DoF on the star).
"""
import numpy as np


class Mesh:
    def __init__(self, M):
        self.M = M
        self.h = 1.0 / M
        n1 = M + 1
        self.n1 = n1
        self.nv = n1 * n1
        v = np.arange(self.nv)
        self.vxy = np.stack([(v % n1) * self.h, (v // n1) * self.h], axis=1)
        cells = []
        for j in range(M):
            for i in range(M):
                a = i + n1 * j
                b = (i + 1) + n1 * j
                c = i + n1 * (j + 1)
                d = (i + 1) + n1 * (j + 1)
                cells.append([a, b, c])
                cells.append([d, c, b])
        self.cells = np.array(cells, dtype=np.int64)
        self.nc = len(cells)
        n2 = 2 * M + 1
        self.n2 = n2
        self.nn = n2 * n2
        g = np.arange(self.nn)
        self.nxy = np.stack([(g % n2) * 0.5 * self.h, (g // n2) * 0.5 * self.h], axis=1)
        vn = 2 * (self.cells % n1) + n2 * 2 * (self.cells // n1)
        gi, gj = vn % n2, vn // n2

        def mid(x, y):
            return (gi[:, x] + gi[:, y]) // 2 + n2 * ((gj[:, x] + gj[:, y]) // 2)

        self.cell_p2 = np.concatenate(
            [vn, mid(1, 2)[:, None], mid(0, 2)[:, None], mid(0, 1)[:, None]], axis=1)
        # free numbering
        gi_all, gj_all = g % n2, g // n2
        interior = (gi_all > 0) & (gi_all < n2 - 1) & (gj_all > 0) & (gj_all < n2 - 1)
        self.node_free = np.full(self.nn, -1, dtype=np.int64)
        self.node_free[interior] = (gi_all[interior] - 1) + (n2 - 2) * (gj_all[interior] - 1)
        self.n_free_nodes = (n2 - 2) ** 2
        self.n_free = 2 * self.n_free_nodes + self.nv
        self.p_offset = 2 * self.n_free_nodes

    # --- DoF helpers -----------------------------------------------------
    def vel_dof(self, node, comp):
        """Free DoF index of (node, comp), or -1 on the Dirichlet boundary."""
        k = self.node_free[node]
        return np.where(k >= 0, 2 * k + comp, -1)

    def p_dof(self, vert):
        return self.p_offset + np.asarray(vert)

    def cell_dofs(self):
        """(nc, 15) free DoF of each local DoF: 6 x-velocity, 6 y-velocity, 3 pressure (-1 = Dirichlet)."""
        ux = self.vel_dof(self.cell_p2, 0)
        uy = self.vel_dof(self.cell_p2, 1)
        p = self.p_dof(self.cells)
        return np.concatenate([ux, uy, p], axis=1)

    def free_node_xy(self):
        idx = np.nonzero(self.node_free >= 0)[0]
        order = np.argsort(self.node_free[idx])
        return self.nxy[idx[order]]

    # --- patches -------------------------------------------------------------
    def patches(self):
        """List (one per vertex) of sorted free DoF indices of the Vanka+star patch."""
        incident = [[] for _ in range(self.nv)]
        for c in range(self.nc):
            for vv in self.cells[c]:
                incident[vv].append(c)
        out = []
        for vv in range(self.nv):
            nodes = np.unique(self.cell_p2[incident[vv]].ravel())
            d = np.concatenate([self.vel_dof(nodes, 0), self.vel_dof(nodes, 1)])
            d = d[d >= 0]
            d = np.concatenate([d, [self.p_dof(vv)]])
            out.append(np.sort(d))
        return out


def full_from_free(mesh, x_free, bc_x, bc_y):
    """Scatter a free spatial vector (n_free, ...) into full arrays
    (ux (nn,...), uy (nn,...), p (nv,...)); boundary nodes take bc_x/bc_y (nn,...)."""
    ux = np.array(bc_x, dtype=float, copy=True)
    uy = np.array(bc_y, dtype=float, copy=True)
    fr = mesh.node_free >= 0
    k = mesh.node_free[fr]
    ux[fr] = x_free[2 * k]
    uy[fr] = x_free[2 * k + 1]
    p = np.array(x_free[mesh.p_offset:], dtype=float, copy=True)
    return ux, uy, p
