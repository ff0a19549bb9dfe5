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
  MS(theta) = cos(pi theta) I - i sin(pi theta) X (x) X.  With phases, the
  printed rows 0-2 are those of exp(-i pi theta P(phi1) (x) P(phi0)), with
  P(phi) = [[0, e^{-2 pi i phi}], [e^{2 pi i phi}, 0]] (the GPI matrix); the
  printed entry (3, 0) carries e^{-2 pi i (phi0 + phi1)}, which makes the
  matrix non-unitary, and is read as e^{+2 pi i (phi0 + phi1)} (MSP below).
* GPI is treated as a parametrized gate (its Appendix A matrix depends on phi).
* Rot(theta, phi, lambda) is Appendix A's single-qubit rotation (radians).  The
  H-Rz decomposition printed for a "general rotation" in Sec. 2.5 describes a
  different gate; it is not used.
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


def ROT(theta, phi, lam):
    """Rot(theta, phi, lambda) of Appendix A."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return _c([[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]])


def MSP(phi0, phi1, theta):
    """MS(phi0, phi1, theta) of Appendix A (phases in turns), entry (3, 0) as read
    above; MSP(0, 0, t) = MS(t)."""
    c, s = np.cos(np.pi * theta), np.sin(np.pi * theta)
    e = lambda a: np.exp(-2j * np.pi * a)
    return _c([[c, 0, 0, -1j * e(phi0 + phi1) * s],
               [0, c, -1j * e(phi1 - phi0) * s, 0],
               [0, -1j * e(phi0 - phi1) * s, c, 0],
               [-1j * e(-(phi0 + phi1)) * s, 0, 0, c]])


# ---- analytic derivatives d U / d param ------------------------------------
def dROT(theta, phi, lam):
    """(dRot/dtheta, dRot/dphi, dRot/dlambda)."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    ep, el, epl = np.exp(1j * phi), np.exp(1j * lam), np.exp(1j * (phi + lam))
    d_t = _c([[-s / 2, -el * c / 2], [ep * c / 2, -epl * s / 2]])
    d_p = _c([[0, 0], [1j * ep * s, 1j * epl * c]])
    d_l = _c([[0, -1j * el * s], [0, 1j * epl * c]])
    return d_t, d_p, d_l


def dMSP(phi0, phi1, theta):
    """dMS(phi0, phi1, theta) / dtheta."""
    c, s = np.cos(np.pi * theta), np.sin(np.pi * theta)
    e = lambda a: np.exp(-2j * np.pi * a)
    p = np.pi
    return _c([[-p * s, 0, 0, -1j * p * e(phi0 + phi1) * c],
               [0, -p * s, -1j * p * e(phi1 - phi0) * c, 0],
               [0, -1j * p * e(phi0 - phi1) * c, -p * s, 0],
               [-1j * p * e(-(phi0 + phi1)) * c, 0, 0, -p * s]])



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


# gates with several parameters: Rot reads (theta, phi, lambda)
N_PARAMS = {"ROT": 3}


def matrix(gate: str, param=None, phases=(0.0, 0.0)):
    """Gate matrix; ``param`` ignored for fixed gates, a 3-sequence for Rot;
    ``phases`` = (phi0, phi1) of MS."""
    if gate in FIXED:
        return FIXED[gate]()
    if gate == "ROT":
        return ROT(*param)
    if gate == "MS" and tuple(phases) != (0.0, 0.0):
        return MSP(phases[0], phases[1], param)
    return PARAM[gate][0](param)


def dmatrices(gate: str, param, phases=(0.0, 0.0)):
    """Derivatives of the matrix, one per parameter of the gate."""
    if gate == "ROT":
        return list(dROT(*param))
    if gate == "MS" and tuple(phases) != (0.0, 0.0):
        return [dMSP(phases[0], phases[1], param)]
    return [PARAM[gate][1](param)]


def dmatrix(gate: str, param):
    return PARAM[gate][1](param)


def generators(gate: str, param, phases=(0.0, 0.0)):
    """Output-side generators G_k = i (dU/dparam_k) U^dagger (Hermitian), one per
    parameter.  With them the derivative of <psi|H|psi> through this gate is
    2 Im <lambda|G_k|psi>, lambda and psi taken at the gate's output."""
    U = matrix(gate, param, phases)
    return [1j * d @ U.conj().T for d in dmatrices(gate, param, phases)]


def generator(gate: str, param):
    """The generator of a one-parameter gate (see generators)."""
    return generators(gate, param)[0]
