"""Labels of integrands with poles of higher order (Eq. (5)), shared by the
oracle pins and the library tests (integer labels only, no arithmetic of the
method)."""
import numpy as np

from ami_inputs import random_self_energy

# a double pole present from the start: (1/beta) sum_nu 1/((i nu + E1)^2 (i nu + i Omega + E2))
DOUBLE = (np.array([[1, 0], [1, 0], [1, 1]]), np.array([[1, 0], [1, 0], [0, 1]]), 1, [1, 0])
# a double pole that appears only after the first sum
LATER = (np.array([[1, 0, 0], [0, 1, 1], [-1, 1, 1]]), np.array([[1, 0], [0, 1], [-1, 1]]), 2, [1, 1, 0])


def repeated_line(order, i, line=0):
    """A generated self-energy with one internal line taken twice (same label,
    same energy): the diagram with a constant self-energy inserted on it,
    whose propagator squared gives poles of second order."""
    d = random_self_energy(order, (0, order, i))
    j = [r for r in range(d.alpha.shape[0]) if np.any(d.alpha[r, :d.n_int])][line]
    return (np.vstack([d.alpha, d.alpha[j:j + 1]]), np.vstack([d.eps, d.eps[j:j + 1]]), d.n_int,
            list(d.fermionic))


# Single sums with poles of order three and four, and with a squared
# denominator that moves under the derivative of another double pole (the
# Leibniz factor (-a)^k C(m+k-1, k) with m >= 2, k >= 1, for a = +1 and -1).
# Each pins a different branch of the Eq. (5) expansion: Taylor leaves T_2 and
# T_3, and moving powers m = 2, 3 with k = 1, 2.
SINGLE_SUM_CASES = {
    # (1/beta) sum 1/((i nu + E1)^3 (i nu + i Omega + E2))
    "triple": (np.array([[1, 0], [1, 0], [1, 0], [1, 1]]), np.array([[1, 0], [1, 0], [1, 0], [0, 1]]), 1, [1, 0]),
    # (1/beta) sum 1/((i nu + E1)^4 (i nu + i Omega + E2))
    "quadruple": (np.array([[1, 0]] * 4 + [[1, 1]]), np.array([[1, 0]] * 4 + [[0, 1]]), 1, [1, 0]),
    # (1/beta) sum 1/((i nu + E1)^2 (i nu + i Omega + E2)^2)
    "square_square": (np.array([[1, 0], [1, 0], [1, 1], [1, 1]]), np.array([[1, 0], [1, 0], [0, 1], [0, 1]]), 1,
                      [1, 0]),
    # (1/beta) sum 1/((i nu + E1)^2 (-i nu + i Omega + E2)^2)
    "square_negsquare": (np.array([[1, 0], [1, 0], [-1, 1], [-1, 1]]), np.array([[1, 0], [1, 0], [0, 1], [0, 1]]),
                         1, [1, 0]),
    # (1/beta) sum 1/((i nu + E1)^3 (i nu + E2)^2), the external slot unused
    "triple_square": (np.array([[1, 0]] * 5), np.array([[1, 0]] * 3 + [[0, 1]] * 2), 1, [1, 0]),
}


CASES = {"double": DOUBLE, "later": LATER, "o3": repeated_line(3, 0), "o4": repeated_line(4, 1),
         "o4b": repeated_line(4, 3, 1), **SINGLE_SUM_CASES}
