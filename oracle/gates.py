"""Gate matrices of the paper's Appendix A, in complex128 (TEST INFRASTRUCTURE).

Conventions
-----------
* Rotation angles (RX, RY, RZ, ZZ) are in radians; the IonQ gates (GPI, GPI2,
  MS) take their phase / angle in turns, as in Appendix A.
* For 2-qubit gates the first wire of the pair is the more significant index
  bit of the 4x4 matrix (the CNOT of Sec. 2.3 with its control first).

Readings of entries the source prints inconsistently
----------------------------------------------------
* ECR (Appendix A, "Fixed gates"): the printed rows 2 and 3 are not the rows of
  a unitary matrix.  The printed rows 0 and 1 are exactly the first two rows of
  (I (x) X - X (x) Y)/sqrt(2), which is unitary and squares to the identity;
  that matrix is used here.
* MS (Appendix A, "Other gates"): for phi0 = phi1 = 0 every reading agrees on
  MS(theta) = cos(pi theta) I - i sin(pi theta) X (x) X; only that case is
  provided.
* GPI is treated as a parametrized gate (its Appendix A matrix depends on phi).
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)
I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)  # Pauli Y (for readings and tests)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _c(a):
    return np.asarray(a, dtype=np.complex128)


# ---- (anti)diagonal gates --------------------------------------------------
def S():
    return _c([[1, 0], [0, 1j]])


def Zg():
    return Z.copy()


def RZ(t):
    return _c([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]])


def CZ():
    return _c(np.diag([1, 1, 1, -1]))


def ZZ(t):
    """Rzz(theta) of Appendix A: diag(e^{-i t/2}, e^{i t/2}, e^{i t/2}, e^{-i t/2})."""
    a, b = np.exp(-0.5j * t), np.exp(0.5j * t)
    return _c(np.diag([a, b, b, a]))


def GPI(phi):
    return _c([[0, np.exp(-2j * np.pi * phi)], [np.exp(2j * np.pi * phi), 0]])


# ---- permutation gates -----------------------------------------------------
def Xg():
    return X.copy()


def SWAP():
    return _c([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]])


def CNOT():
    return _c([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])


# ---- fixed gates -----------------------------------------------------------
def H():
    return _c([[1, 1], [1, -1]]) / SQ2


def SX():
    return 0.5 * _c([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])


def ECR():
    """(I (x) X - X (x) Y) / sqrt(2): rows [0,1,0,i], [1,0,-i,0], [0,i,0,1], [-i,0,1,0]."""
    return _c([[0, 1, 0, 1j], [1, 0, -1j, 0], [0, 1j, 0, 1], [-1j, 0, 1, 0]]) / SQ2


# ---- rotations -------------------------------------------------------------
def RX(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return _c([[c, -1j * s], [-1j * s, c]])


def RY(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return _c([[c, -s], [s, c]])


def GPI2(phi):
    return _c([[1, -1j * np.exp(-2j * np.pi * phi)], [-1j * np.exp(2j * np.pi * phi), 1]]) / SQ2


def MS(t):
    """MS(0, 0, theta): cos(pi t) on the diagonal, -i sin(pi t) on the anti-diagonal."""
    c, s = np.cos(np.pi * t), np.sin(np.pi * t)
    return _c([[c, 0, 0, -1j * s], [0, c, -1j * s, 0], [0, -1j * s, c, 0], [-1j * s, 0, 0, c]])


# ---- analytic derivatives d U / d param ------------------------------------
def dRX(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return _c([[-s / 2, -0.5j * c], [-0.5j * c, -s / 2]])


def dRY(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return _c([[-s / 2, -c / 2], [c / 2, -s / 2]])


def dRZ(t):
    return _c([[-0.5j * np.exp(-0.5j * t), 0], [0, 0.5j * np.exp(0.5j * t)]])


def dZZ(t):
    a, b = -0.5j * np.exp(-0.5j * t), 0.5j * np.exp(0.5j * t)
    return _c(np.diag([a, b, b, a]))


def dGPI(phi):
    w = 2j * np.pi
    return _c([[0, -w * np.exp(-w * phi)], [w * np.exp(w * phi), 0]])


def dGPI2(phi):
    w = 2j * np.pi
    return _c([[0, -2 * np.pi * np.exp(-w * phi)], [2 * np.pi * np.exp(w * phi), 0]]) / SQ2


def dMS(t):
    c, s = np.cos(np.pi * t), np.sin(np.pi * t)
    p = np.pi
    return _c([[-p * s, 0, 0, -1j * p * c], [0, -p * s, -1j * p * c, 0],
               [0, -1j * p * c, -p * s, 0], [-1j * p * c, 0, 0, -p * s]])


FIXED = {"H": H, "X": Xg, "Z": Zg, "S": S, "SX": SX, "CNOT": CNOT, "CZ": CZ,
         "SWAP": SWAP, "ECR": ECR}
PARAM = {"RX": (RX, dRX), "RY": (RY, dRY), "RZ": (RZ, dRZ), "GPI": (GPI, dGPI),
         "GPI2": (GPI2, dGPI2), "ZZ": (ZZ, dZZ), "MS": (MS, dMS)}


def matrix(gate: str, param=None):
    """Gate matrix; ``param`` ignored for fixed gates."""
    if gate in FIXED:
        return FIXED[gate]()
    return PARAM[gate][0](param)


def dmatrix(gate: str, param):
    return PARAM[gate][1](param)


def generator(gate: str, param):
    """Output-side generator G = i (dU/dparam) U^dagger (Hermitian).

    With it the derivative of <psi|H|psi> through this gate is
    2 Im <lambda|G|psi>, lambda and psi taken at the gate's output."""
    U = matrix(gate, param)
    return 1j * dmatrix(gate, param) @ U.conj().T
