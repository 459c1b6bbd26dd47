"""Write tests/golden/oracle_tiny.json: the FP64 oracle's Gram, shift, factor,
R, image and SRF diagonal for two tiny seeded encodings (a 3 x 2 grid with two
coils and two species plus off-resonance; an underdetermined 4 x 3 grid), to
12 significant digits.

The values come from oracle/ alone (run: python tests/golden/make_golden.py).
They pin the oracle against unnoticed drift in its conventions (sign, index
order, shift, conjugation): tests/test_oracle_pins.py recomputes them."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2410_06129_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_tiny.json")


def cases():
    rng = np.random.default_rng(2410)
    k1 = rng.uniform(-1.5, 1.5, size=(7, 2))
    e1 = synth.Encoding(3, 2, k1, t=synth.sample_times(7, 1e-3), coil=synth.coil_maps(3, 2, 2, rng),
                        b0_hz=synth.b0_map(3, 2, rng), species_hz=np.array([0.0, 60.0]))
    k2 = rng.uniform(-2.0, 2.0, size=(5, 2))
    e2 = synth.Encoding(4, 3, k2, coil=synth.coil_maps(4, 3, 2, rng))
    return {"overdetermined_species_b0": e1, "underdetermined": e2}


def enc_record(e):
    return {"nx": e.nx, "ny": e.ny, "k": e.k.tolist(),
            "t": None if e.t is None else e.t.tolist(),
            "coil": None if e.coil is None else np.stack([e.coil.real, e.coil.imag], -1).tolist(),
            "b0_hz": None if e.b0_hz is None else e.b0_hz.tolist(),
            "species_hz": None if e.species_hz is None else e.species_hz.tolist()}


def cplx(a):
    a = np.asarray(a)
    return np.stack([a.real, a.imag], -1).round(12).tolist()


def compute(name, e):
    rng = np.random.default_rng(7)
    d = rng.standard_normal((2, e.M)) + 1j * rng.standard_normal((2, e.M))
    if e.M >= e.N:
        b = oracle.Build(e, rel=1e-2)
        R = b.recon_matrix()
        L, G = b.L, b.G
    else:
        b = oracle.RightBuild(e, rel=1e-2)
        R = b.recon_matrix()
        L, G = b.L, b.Gr
    E = oracle.encoding_matrix(e)
    return {"lam": round(b.lam, 14), "G": cplx(G), "L": cplx(L), "R": cplx(R), "d": cplx(d),
            "x": cplx(b.reconstruct(d)), "srf_diag": cplx(np.diagonal(oracle.srf_matrix(R, E)))}


def main():
    rec = {"source": "oracle/pinv_oracle.py via tests/golden/make_golden.py", "cases": {}}
    for name, e in cases().items():
        rec["cases"][name] = {"encoding": enc_record(e), "values": compute(name, e)}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
