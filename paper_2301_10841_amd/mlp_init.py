"""Initial weights of the chooser's perceptron (He-normal weights, zero
biases), as one float32 vector in the library's parameter order: W1
(in_dim x hidden, row-major), b1, W2 (hidden x hidden), b2, W3 (hidden), b3."""

import numpy as np


def he_init(rng: np.random.Generator, in_dim: int, hidden: int) -> np.ndarray:
    w1 = rng.normal(0.0, np.sqrt(2.0 / in_dim), size=(in_dim, hidden))
    w2 = rng.normal(0.0, np.sqrt(2.0 / hidden), size=(hidden, hidden))
    w3 = rng.normal(0.0, np.sqrt(1.0 / hidden), size=hidden)
    return np.concatenate([w1.ravel(), np.zeros(hidden), w2.ravel(), np.zeros(hidden), w3, [0.0]]).astype(np.float32)
