"""Single-qubit matrices of the extended operator alphabet.

Methods, Qubit Hamiltonians: the alphabet is ``[Z, 0, 1, X, Y, -, +] -> [0..6]`` where codes
above 2 are off-diagonal.  Matrices are written in the computational basis ``(|0>, |1>)``;
entry ``[r, c] = <r|W|c>``.

* ``0 = |0><0|`` and ``1 = |1><1|`` are the projectors (Supplemental Table S1 defines them as
  ``f f^dagger`` and ``f^dagger f``).
* ``- = |0><1|`` is the qubit image of the annihilator: ``f_j = 1/2 (X_j + i Y_j) Z...``
  (Methods, Fermionic Hamiltonians), and ``1/2 (X + iY) = |0><1|``.
* ``+ = |1><0|`` is its adjoint.
"""
import numpy as np

CODES = {"Z": 0, "0": 1, "1": 2, "X": 3, "Y": 4, "-": 5, "+": 6}
LETTERS = {v: k for k, v in CODES.items()}

I2 = np.eye(2, dtype=np.complex128)
MATS = np.zeros((7, 2, 2), dtype=np.complex128)
MATS[0] = [[1, 0], [0, -1]]  # Z
MATS[1] = [[1, 0], [0, 0]]  # |0><0|
MATS[2] = [[0, 0], [0, 1]]  # |1><1|
MATS[3] = [[0, 1], [1, 0]]  # X
MATS[4] = [[0, -1j], [1j, 0]]  # Y
MATS[5] = [[0, 1], [0, 0]]  # |0><1|
MATS[6] = [[0, 0], [1, 0]]  # |1><0|


def is_offdiagonal(code: int) -> bool:
    return code > 2


def mat(code: int) -> np.ndarray:
    return MATS[int(code)]
