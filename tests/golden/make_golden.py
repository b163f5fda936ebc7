"""Write the stored oracle references under tests/golden/.

    python tests/golden/make_golden.py            (from the repository root)

For each small workload below, the seeded inputs come from synth/ and every
value from the CPU FP64 oracle (oracle/), nothing else: the plane-wave matrix
elements M_vc(q+G) of the spin-summed product (arXiv:2206.00808, Sec. II, Eq.
(matrix_el)), the polarizability chi0_GG'(q, i omega) of the Adler-Wiser band
sum on the imaginary axis (Sec. II), and eps^-1 for eps = I - v chi0 (Sec. II).
A file is named and keyed by the workload's parameter digest
(synth.config_digest), so a changed workload no longer matches its stored file.

Stored per file: a seeded sample of M entries, every diagonal entry and the
whole first row of chi0 and eps^-1 per frequency, a seeded sample of their
off-diagonal entries, and the Frobenius norms. Values are printed with 17
significant digits (exact round trip of binary64).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

WORKLOADS = {
    # the smallest workload: 16^3 box, 8 x 32 pairs, 59 eps-sphere G, static
    "C1": "FFT box 16x16x16, N_v 8, N_c 32, 59 eps-sphere G, static",
    # an elongated box, whose transforms run on xy-planes first and z last
    "T4": "FFT box 16x16x40, N_v 5, N_c 21, static and one imaginary frequency",
}

N_M = 48       # sampled matrix elements per file
N_OFF = 32     # sampled off-diagonal chi0 / eps^-1 entries per frequency


def path_for(name):
    cfg = synth.CONFIGS[name]
    return os.path.join(HERE, f"{name}_{synth.config_digest(cfg)}.txt")


def reference(name):
    """The oracle's M, chi0 and eps^-1 for the workload (complex128)."""
    s = synth.build_system(synth.CONFIGS[name])
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    return s, m, x, e


def _sample(name, m, n):
    """Seeded sample indices: M entries (v, c, G), and off-diagonal (G, G')."""
    rng = np.random.default_rng(1000 + synth.CONFIGS[name].seed)
    nv, nc, ng = m.shape
    mi = np.stack([rng.integers(0, nv, N_M), rng.integers(0, nc, N_M),
                   rng.integers(0, ng, N_M)], axis=1)
    # the G = 0 (head) entry of the first four sampled pairs
    mi[:4, 2] = 0
    off = []
    while len(off) < N_OFF:
        i, j = (int(a) for a in rng.integers(0, n, 2))
        if i != j and (i, j) not in off:
            off.append((i, j))
    return mi, np.asarray(off)


def write(name):
    s, m, x, e = reference(name)
    n = len(s["geps"])
    mi, off = _sample(name, m, n)
    cfg = synth.CONFIGS[name]
    lines = [
        f"# Stored CPU FP64 oracle reference, workload {name}: {WORKLOADS[name]}.",
        f"# digest {synth.config_digest(cfg)}  (synth.config_digest of the workload's parameters)",
        "# Written by tests/golden/make_golden.py from oracle/ and synth/ only.",
        "# M: plane-wave matrix element M_vc(q+G) (arXiv:2206.00808, Sec. II, Eq. (matrix_el));",
        "# chi0: Adler-Wiser polarizability at imaginary frequency (Sec. II); epsinv: (I - v chi0)^-1.",
        "# Lines: 'M v c G re im' | 'chi0 f i j re im' | 'epsinv f i j re im' | 'norm kind f value'.",
        f"shape {m.shape[0]} {m.shape[1]} {n} {len(s['omega'])}",
    ]
    fmt = lambda z: f"{z.real:.17g} {z.imag:.17g}"  # noqa: E731
    for v, c, g in mi:
        lines.append(f"M {v} {c} {g} {fmt(m[v, c, g])}")
    for f in range(len(s["omega"])):
        ent = [(i, i) for i in range(n)] + [(0, j) for j in range(1, n)] + \
              [(int(i), int(j)) for i, j in off]
        for kind, a in (("chi0", x[f]), ("epsinv", e[f])):
            for i, j in ent:
                lines.append(f"{kind} {f} {i} {j} {fmt(a[i, j])}")
            lines.append(f"norm {kind} {f} {np.linalg.norm(a):.17g}")
    with open(path_for(name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path_for(name)


def read(path):
    """Parse a stored reference: {'shape': (...), 'M': {(v,c,G): z},
    'chi0'/'epsinv': {(f,i,j): z}, 'norm': {(kind,f): value}}."""
    out = {"M": {}, "chi0": {}, "epsinv": {}, "norm": {}}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0] == "shape":
                out["shape"] = tuple(int(a) for a in t[1:])
            elif t[0] == "M":
                out["M"][tuple(int(a) for a in t[1:4])] = complex(float(t[4]), float(t[5]))
            elif t[0] in ("chi0", "epsinv"):
                out[t[0]][tuple(int(a) for a in t[1:4])] = complex(float(t[4]), float(t[5]))
            elif t[0] == "norm":
                out["norm"][(t[1], int(t[2]))] = float(t[3])
    return out


if __name__ == "__main__":
    for name in WORKLOADS:
        print(write(name))
