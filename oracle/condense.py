"""Static condensation, Section 4.1.2 (test infrastructure; see package header).

Both strategies are written exactly as the Schur complements of the paper,
with dense solves of the eliminated blocks (no factorisation tricks):

* v-cond, eq. ST.1: eliminate the cell velocities U_T; the globally coupled
  unknowns of T are (U_dT, P_T).
* v&p-cond, eq. ST.2: eliminate U_T and the non-mean pressure modes; the
  globally coupled unknowns are (U_dT, mean pressure).

Reading: the right-hand side of eq. zero-residual.T writes 0 for the rows of
the non-mean pressure modes, while eq. def:HHOAB puts the Dirichlet mass datum
Ghat in every pressure row.  The residual definition is followed: those rows
carry the non-mean part of Ghat (it vanishes for homogeneous Dirichlet data).
"""
from __future__ import annotations

import numpy as np

from .hho import LocalHHO, vector_system


def condense_v(L: LocalHHO):
    """(S, rhs) of eq. ST.1, unknown order [U_dT (face, comp, mode); P_T (nT)]."""
    A_TT, A_Td, A_dd, B_T, B_d, F_T, G_d, Gh = vector_system(L)
    nP = L.nT
    top = np.block([[A_dd, B_d.T], [B_d, np.zeros((nP, nP))]])
    left = np.vstack([A_Td.T, B_T])                  # [A_dT; B_TT]
    right = np.hstack([A_Td, B_T.T])                 # [A_Td, B_TT^T]
    S = top - left @ np.linalg.solve(A_TT, right)
    rhs = np.concatenate([G_d, Gh]) - left @ np.linalg.solve(A_TT, F_T)
    return S, rhs


def condense_vp(L: LocalHHO):
    """(S, rhs) of eq. ST.2, unknown order [U_dT (face, comp, mode); mean pressure]."""
    A_TT, A_Td, A_dd, B_T, B_d, F_T, G_d, Gh = vector_system(L)
    Bb_T, Bt_T = B_T[:1], B_T[1:]
    Bb_d, Bt_d = B_d[:1], B_d[1:]
    nt = Bt_T.shape[0]
    M = np.block([[A_TT, Bt_T.T], [Bt_T, np.zeros((nt, nt))]])
    top = np.block([[A_dd, Bb_d.T], [Bb_d, np.zeros((1, 1))]])
    left = np.block([[A_Td.T, Bt_d.T], [Bb_T, np.zeros((1, nt))]])
    right = np.block([[A_Td, Bb_T.T], [Bt_d, np.zeros((nt, 1))]])
    S = top - left @ np.linalg.solve(M, right)
    rhs = np.concatenate([G_d, Gh[:1]]) - left @ np.linalg.solve(M, np.concatenate([F_T, Gh[1:]]))
    return S, rhs


def recover_v(L: LocalHHO, Ud: np.ndarray, P: np.ndarray):
    """Cell velocities from the v-cond unknowns (first block row of eq. def:HHOAB)."""
    A_TT, A_Td, _, B_T, _, F_T, _, _ = vector_system(L)
    return np.linalg.solve(A_TT, F_T - A_Td @ Ud - B_T.T @ P)


def recover_vp(L: LocalHHO, Ud: np.ndarray, Pbar: float):
    """(U_T, full pressure) from the v&p-cond unknowns (top block of eq. zero-residual.T)."""
    A_TT, A_Td, _, B_T, B_d, F_T, _, Gh = vector_system(L)
    Bb_T, Bt_T, Bt_d = B_T[:1], B_T[1:], B_d[1:]
    nt = Bt_T.shape[0]
    M = np.block([[A_TT, Bt_T.T], [Bt_T, np.zeros((nt, nt))]])
    r = np.concatenate([F_T - A_Td @ Ud - Bb_T.T @ np.atleast_1d(Pbar), Gh[1:] - Bt_d @ Ud])
    y = np.linalg.solve(M, r)
    nU = A_TT.shape[0]
    return y[:nU], np.concatenate([np.atleast_1d(Pbar), y[nU:]])
