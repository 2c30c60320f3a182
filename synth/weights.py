"""Seeded random parameters of the learned scorer (an input generator: no
arithmetic of the method lives here).

Flat FP32 vector in the scorer's order W1[64][40], b1[64], W2[64][64], b2[64],
w3[64], b3; weights drawn with He-style scales, biases zero unless asked.
"""
import numpy as np

N_IN, N_H = 40, 64
N_PARAM = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def random_params(rng: np.random.Generator, scale: float = 1.0, bias: float = 0.0) -> np.ndarray:
    w1 = rng.normal(0.0, scale * np.sqrt(2.0 / N_IN), N_H * N_IN)
    w2 = rng.normal(0.0, scale * np.sqrt(2.0 / N_H), N_H * N_H)
    w3 = rng.normal(0.0, scale * np.sqrt(1.0 / N_H), N_H)
    b = [rng.normal(0.0, bias, n) if bias > 0 else np.zeros(n) for n in (N_H, N_H, 1)]
    return np.concatenate([w1, b[0], w2, b[1], w3, b[2]]).astype(np.float32)
