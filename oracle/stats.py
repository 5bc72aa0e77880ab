"""O4: Porter-Thomas statistics of output probabilities.

For deep random circuits the scaled probabilities x = 2^N |<tau|psi>|^2 follow
the exponential (Porter-Thomas) law the paper compares against in Fig. 2
(log-transformed there).  Closed forms for x ~ Exp(1): E[x] = 1 (exact over
all bitstrings, by normalisation), E[x^2] = 2 (2 * 2^N / (2^N + 1) over the
full distribution of a Haar state), E[-ln x] = Euler's gamma, and y = ln x has
density exp(y - e^y).
"""
import numpy as np
from scipy import stats as st

EULER_GAMMA = 0.5772156649015329


def scaled_probabilities(amps: np.ndarray, n_qubits: int) -> np.ndarray:
    return (2.0 ** n_qubits) * np.abs(np.asarray(amps)) ** 2


def porter_thomas_summary(x: np.ndarray) -> dict:
    x = np.asarray(x, dtype=np.float64)
    pos = x[x > 0]
    ks = st.kstest(x, "expon")
    return {
        "n": int(x.size),
        "mean": float(np.mean(x)),
        "second_moment": float(np.mean(x * x)),
        "mean_neg_log": float(np.mean(-np.log(pos))),
        "ks_statistic": float(ks.statistic),
        "ks_pvalue": float(ks.pvalue),
    }


def log_pt_density(y: np.ndarray) -> np.ndarray:
    """Density of y = ln x for x ~ Exp(1)."""
    return np.exp(y - np.exp(y))
