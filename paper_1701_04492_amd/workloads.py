"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Random draws only -- none of the method's arithmetic lives here.  numpy
Generator(PCG64(seed)), draws in the order listed.  Workload i uses seed
SEED0 + i.

1  1-D type II, N = 1024, iid x on [0,1), c complex128 N(0,1), eps 1e-12, FP64 plain path.
2  1-D type II and type I, N = 2^20, c N(0,1), x jittered (j + U(-1/2,1/2))/N or iid U[0,1);
   eps 1e-12 FP64, eps 1e-6 FP32.
3  forward + backward, N = 2^22, complex64, iid x, y complex N(0,1); FD/oracle check at N = 4096.
4  512 type-II transforms, N_b = round(2^U(8,16)), then per b: x iid, c N(0,1); eps 1e-6 FP32.
5  2-D type II, 1024 x 1024 coefficients, M = 2^20 points at radius 0.5 U, angle 2 pi U around
   (1/2, 1/2); eps 1e-6 FP32.
The paper's experiments are themselves synthetic (Gaussian coefficients, uniform and
"worst grid" samples, Sec. 2.4); no dataset stands behind these workloads.
"""
import numpy as np

SEED0 = 1701044920


def rng_for(workload):
    return np.random.Generator(np.random.PCG64(SEED0 + int(workload)))


def complex_normal(rng, n):
    """Real block first, then imaginary block."""
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def iid_samples(rng, m):
    return rng.random(m)


def jittered_samples(rng, n):
    return (np.arange(n) + rng.uniform(-0.5, 0.5, n)) / n


def worst_grid(n, gamma):
    """Sec. 2.4: x_j = (j + gamma)/N for j <= N/2, (j - gamma)/N otherwise."""
    j = np.arange(n)
    return np.where(j <= n // 2, (j + gamma) / n, (j - gamma) / n)


def type2_case(workload, n, m=None, dist="iid"):
    rng = rng_for(workload)
    m = n if m is None else m
    c = complex_normal(rng, n)
    x = iid_samples(rng, m) if dist == "iid" else jittered_samples(rng, n)
    return x, c


def batch_case(workload=4, batch=512, lo=8.0, hi=16.0):
    rng = rng_for(workload)
    Ns = np.rint(2.0 ** rng.uniform(lo, hi, batch)).astype(np.int64)
    xs, cs = [], []
    for n in Ns:
        xs.append(iid_samples(rng, int(n)))
        cs.append(complex_normal(rng, int(n)))
    return Ns, xs, cs


def polar_case(workload=5, n1=1024, n2=1024, m=1 << 20):
    rng = rng_for(workload)
    C = complex_normal(rng, n1 * n2).reshape(n1, n2)
    r = 0.5 * rng.random(m)
    th = 2.0 * np.pi * rng.random(m)
    return 0.5 + r * np.cos(th), 0.5 + r * np.sin(th), C
