"""D3Q19 velocity set in the population order of the library interface
(rest, the six axis links, then the twelve diagonals; odd q has its opposite at
q + 1), written out for the tests' own moment and symmetry checks."""
import numpy as np

C = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=np.int64)


def opposite(q):
    return int(np.nonzero((C == -C[q]).all(axis=1))[0][0])


def index_of(c):
    return int(np.nonzero((C == np.asarray(c)).all(axis=1))[0][0])
