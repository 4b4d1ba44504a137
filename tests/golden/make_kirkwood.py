"""Write kirkwood.txt: energies of a point charge q at distance b from the centre
of a dielectric sphere (radius a, permittivity eps_in) in a screened solvent
(eps_out, kappa), from the classical Kirkwood series

  E(b) = q^2/2 sum_n b^{2n}/a^{2n+1} ((n+1) + (eps_out/eps_in) g_n) / (eps_in n - eps_out g_n),
  g_n = z k_n'(z)/k_n(z), z = kappa a,

summed in 40-digit arithmetic, together with dE/db.  This is the continuous
model that the discrete ddLPB energy approximates (Sec. 1, LPB equation)."""
import os

import mpmath as mp

mp.mp.dps = 40


def kn(n, z):
    return mp.sqrt(mp.pi / (2 * z)) * mp.besselk(n + mp.mpf(1) / 2, z)


def kirkwood(q, a, b, e1, e2, kap, nmax=80):
    a, b, e1, e2, kap, q = map(mp.mpf, (a, b, e1, e2, kap, q))
    z = kap * a
    E = mp.mpf(0)
    dE = mp.mpf(0)
    for n in range(nmax):
        g = z * (-kn(n + 1, z) + n / z * kn(n, z)) / kn(n, z)
        c = ((n + 1) + (e2 / e1) * g) / (e1 * n - e2 * g) / a ** (2 * n + 1)
        E += b ** (2 * n) * c
        if n > 0:
            dE += 2 * n * b ** (2 * n - 1) * c
    return q * q / 2 * E, q * q / 2 * dE


CASES = [  # q, a, b, eps_in, eps_out, kappa
    (1.0, 3.0, 0.9, 1.0, 78.54, 0.104),
    (-0.7, 2.5, 1.0, 2.0, 78.54, 0.104),
    (0.5, 4.0, 1.6, 1.0, 40.0, 0.3),
]

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kirkwood.txt")
    with open(out, "w") as fh:
        fh.write("# q a b eps_in eps_out kappa E dE_db   (e^2/A, e^2/A^2)\n")
        for c in CASES:
            E, dE = kirkwood(*c)
            fh.write(" ".join(repr(float(v)) for v in c) + " %s %s\n" % (mp.nstr(E, 20), mp.nstr(dE, 20)))
    print(open(out).read())
