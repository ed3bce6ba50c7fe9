"""D3Q19 velocity set (paper Sec. II.B, Table I).

Index 0 is the rest velocity (the paper's i = 1), indices 1-6 the six
axis neighbours (paper i = 2..7, weight 1/18) and 7-18 the twelve
face-diagonal neighbours (paper i = 8..19, weight 1/36).  The paper fixes
the shells but not the order inside a shell; the order below is one fixed
choice (reading R21).  Results do not depend on it except through the
order of floating-point sums.
"""

import numpy as np

C = np.array(
    [
        [0, 0, 0],
        [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
        [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
        [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
        [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
    ],
    dtype=np.int64,
)

W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=np.float64)

# opposite direction: C[OPP[i]] == -C[i]
OPP = np.array(
    [int(np.nonzero((C == -C[i]).all(axis=1))[0][0]) for i in range(19)], dtype=np.int64
)

CS2 = 1.0 / 3.0  # c_s^2 with dx = dt = 1 (Sec. II.B, Step 1)

Q = 19
