"""Dense matrix statements of the refinement method, for pinning the oracle on
tiny inputs.  These follow the paper's matrix form, not the oracle's loops:
Section 3.3 states the sweep as SOR on L z = 0 with L = D - A the Laplacian
of the star expansion H* (weighted degree on the diagonal).  A relaxed Jacobi
step on L z = 0 is z <- z - omega D^{-1} L z."""
import numpy as np


def star_adjacency(n_nodes, n_edges, eptr, eidx, w=None):
    """Symmetric weighted adjacency A of H* (nodes first, then hyperedges):
    A[v, n+e] = A[n+e, v] = w_e for every member v of e (Section 1.1)."""
    R = n_nodes + n_edges
    A = np.zeros((R, R))
    for e in range(n_edges):
        we = 1.0 if w is None else float(w[e])
        for j in range(eptr[e], eptr[e + 1]):
            v = int(eidx[j])
            A[v, n_nodes + e] = we
            A[n_nodes + e, v] = we
    return A


def jacobi_matrix(A, omega):
    """M with z_new = M z_old: I - omega D^{-1} (D - A) on rows with D > 0,
    identity on rows without neighbours."""
    Dg = A.sum(axis=1)
    L = np.diag(Dg) - A
    R = A.shape[0]
    M = np.eye(R)
    nz = Dg > 0
    M[nz] = np.eye(R)[nz] - omega * (L[nz] / Dg[nz, None])
    return M


def edge_first_matrix(A, omega, n_nodes):
    """Hyperedge rows relaxed first (reading old node rows), then node rows
    (reading the new hyperedge rows): the product of two partial relaxations."""
    M = jacobi_matrix(A, omega)
    R = A.shape[0]
    PE = np.eye(R)
    PE[n_nodes:] = M[n_nodes:]
    PV = np.eye(R)
    PV[:n_nodes] = M[:n_nodes]
    return PV @ PE


def projection_matrix(rowmap, rows_coarse):
    P = np.zeros((len(rowmap), rows_coarse))
    P[np.arange(len(rowmap)), rowmap] = 1.0
    return P
