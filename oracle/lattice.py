"""D2Q9 lattice, MRT transformation matrix and selective-filter coefficients.

Sources (arXiv:1812.02459):
* discrete velocities: eq:D2Q9 (Sec. 3.1) -- c_i = (cos((i-1)pi/2), sin((i-1)pi/2))
  for i=1..4 and sqrt(2)(cos((i-5)pi/2+pi/4), sin(...)) for i=5..8;
* weights: Sec. 3.1, text after eq:D2Q9.  The paper prints "omega_{1..8}=1/36";
  read as omega_{5..8}=1/36 so that the weights sum to one;
* sound speed c_s^2 = 1/3, dx = dt = 1 (Sec. 3.1);
* transformation matrix M: eq:D2Q9MRT, copied as printed;
* explicit selective-filter coefficients d_0..d_5: App. B table.
"""

import math

# eq:D2Q9, evaluated from its trigonometric definition and rounded to integers.
C = []
for _i in range(9):
    if _i == 0:
        C.append((0, 0))
    elif _i <= 4:
        _a = (_i - 1) * math.pi / 2
        C.append((int(round(math.cos(_a))), int(round(math.sin(_a)))))
    else:
        _a = (_i - 5) * math.pi / 2 + math.pi / 4
        C.append((int(round(math.sqrt(2) * math.cos(_a))),
                  int(round(math.sqrt(2) * math.sin(_a)))))
C = tuple(C)

# opposite direction: c_opp(i) = -c_i
OPP = tuple(C.index((-cx, -cy)) for (cx, cy) in C)

# weights (Sec. 3.1, with the 1/36 typo read as omega_5..8)
W = (4 / 9,) + (1 / 9,) * 4 + (1 / 36,) * 4

# eq:D2Q9MRT as printed
M = (
    (1, 1, 1, 1, 1, 1, 1, 1, 1),
    (-4, -1, -1, -1, -1, 2, 2, 2, 2),
    (4, -2, -2, -2, -2, 1, 1, 1, 1),
    (0, 1, 0, -1, 0, 1, -1, -1, 1),
    (0, -2, 0, 2, 0, 1, -1, -1, 1),
    (0, 0, 1, 0, -1, 1, 1, -1, -1),
    (0, 0, -2, 0, 2, 1, 1, -1, -1),
    (0, 1, -1, 1, -1, 0, 0, 0, 0),
    (0, 0, 0, 0, 0, 1, -1, 1, -1),
)

# Row norms: the rows of M are mutually orthogonal, so M M^T = diag(MM_DIAG)
# and M^{-1} = M^T diag(1/MM_DIAG).  The orthogonality is checked by a test.
MM_DIAG = tuple(sum(M[k][j] * M[k][j] for j in range(9)) for k in range(9))
MM_DIAG_INV = tuple(1.0 / d for d in MM_DIAG)

# App. B: explicit centred selective filters, coefficients d_0 .. d_{P}
FILTER_D = {
    5: (6 / 16, -4 / 16, 1 / 16),
    7: (5 / 16, -15 / 64, 3 / 32, -1 / 64),
    9: (0.243527493120, -0.204788880640, 0.120007591680, -0.045211119360,
        0.008228661760),
    11: (0.215044884112, -0.187772883589, 0.123755948787, -0.059227575576,
         0.018721609157, -0.002999540835),
}
