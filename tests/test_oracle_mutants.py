"""Planted mistakes in the oracle: each must fail at least one CPU pin.

A pin only pins what a plausible mistake would move. This test copies the
oracle's source, plants one mistake per copy (a dropped term, a wrong sign, a
wrong index, a transposed operand), builds each copy with the oracle's compiler
options (at -O1, which builds faster) into a temporary directory, and runs the
pins of the transport, the local source and the whole step against it (the oracle wrapper loads the
library named by RHD_ORACLE_LIB). Every planted mistake must make some pin fail;
the unmodified source, built and run the same way, must pass them all.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rhd_oracle.cpp")
PINS = ["tests/test_oracle_transport.py", "tests/test_oracle_source.py",
        "tests/test_oracle_step.py"]

# (name, text in the oracle, replacement)
MUTANTS = [
    # transverse axes of the transport (Sec. 3.3, Sec. 4.3)
    ("speed of x on every axis", "S smax_ = ch * ssqrt(smax(Dm[d][d], Dp[d][d]));",
     "S smax_ = ch * ssqrt(smax(Dm[0][0], Dp[0][0]));"),
    ("speed of one side from x", "S smax_ = ch * ssqrt(smax(Dm[d][d], Dp[d][d]));",
     "S smax_ = ch * ssqrt(smax(Dm[d][d], Dp[0][0]));"),
    ("energy flux from F_x", "phim[0] = (ch / c) * Um[1 + d];", "phim[0] = (ch / c) * Um[1];"),
    ("flux row of x on every axis", "phim[1 + k] = c * ch * Um[0] * Dm[d][k];",
     "phim[1 + k] = c * ch * Um[0] * Dm[0][k];"),
    ("mirror flips F_x on every axis", "if (flip && r == 1 + d) v = -v;",
     "if (flip && r == 1) v = -v;"),
    ("z lines mapped transposed", "return g.idx(a, b, t);\n        };\n        // extended line",
     "return g.idx(b, a, t);\n        };\n        // extended line"),
    # transport arithmetic
    ("HLL dissipation sign", "- S(0.5) * (q == 0 ? eps : S(1.0)) * smax_ * (Up[q] - Um[q]);",
     "+ S(0.5) * (q == 0 ? eps : S(1.0)) * smax_ * (Up[q] - Um[q]);"),
    ("eps applied to the F rows too", "- S(0.5) * (q == 0 ? eps : S(1.0)) * smax_",
     "- S(0.5) * eps * smax_"),
    ("PPM left interface sign", "aL = S(0.5) * (a[1] + ai) - (dm0 - dmm) / S(6.0);",
     "aL = S(0.5) * (a[1] + ai) + (dm0 - dmm) / S(6.0);"),
    ("M1 numerator", "chi = (S(3.0) + S(4.0) * f2) /", "chi = (S(3.0) + S(3.0) * f2) /"),
    # PPM limiter (CW84) on non-smooth data
    ("PPM flattening at an extremum dropped", "if ((aR - ai) * (ai - aL) <= S(0.0)) {",
     "if (false) {"),
    ("PPM overshoot cap on the wrong edge", "aL = S(3.0) * ai - S(2.0) * aR;",
     "aR = S(3.0) * ai - S(2.0) * aL;"),
    ("MC slope kept across an extremum", "if ((ap - a0) * (a0 - am) > S(0.0)) {", "if (true) {"),
    ("divergence sign", "s[(int64_t)r * g.N + c] = s[(int64_t)r * g.N + c] - div;",
     "s[(int64_t)r * g.N + c] = s[(int64_t)r * g.N + c] + div;"),
    # local implicit source (Sec. 3.3)
    ("energy recovery ratio inverted", "Enew = E0 - (ch / c) * (Egas - Eg0) + Ssrc;",
     "Enew = E0 - (c / ch) * (Egas - Eg0) + Ssrc;"),
    ("(2 chi_E - chi_F) v.F term sign", "Cc = (S(2.0) * chiE - chiF) * vF / (c * c);",
     "Cc = (S(2.0) * chiE + chiF) * vF / (c * c);"),
    ("order-1 flux denominator", "Fnew[k] = num / (S(1.0) + ch * chiF * tau);",
     "Fnew[k] = num / (S(1.0) + S(2.0) * ch * chiF * tau);"),
    ("order-2 flux: beta^2/2 sign",
     "const S a = S(1.0) + ch * chiF * (S(1.0) + S(0.5) * beta2) * tau;",
     "const S a = S(1.0) + ch * chiF * (S(1.0) - S(0.5) * beta2) * tau;"),
    ("momentum update sign", "Pnew[k] = P0[k] - (Fnew[k] - F0[k]) / (c * ch);",
     "Pnew[k] = P0[k] + (Fnew[k] - F0[k]) / (c * ch);"),
    ("emission without T^4", "S A = chiP * ar * (T2 * T2) * Afac;", "S A = chiP * ar * (T2 * T) * Afac;"),
    ("flux update drops the Doppler term D v",
     "bx[i] = F0[i] + ch * tau * (chiP * Bn * v[i] + chiF * Enew * Dv[i] + (chiF - chiE) * Enew * v[i]);",
     "bx[i] = F0[i] + ch * tau * (chiP * Bn * v[i] + (chiF - chiE) * Enew * v[i]);"),
    # c / chat mix-ups (Sec. 3.1: the reduced speed enters the transport and the
    # R / (tau chat) exchange, the true c the v/c terms and the closure)
    ("beta^2 over c chat", "const S beta2 = v2 / (c * c);", "const S beta2 = v2 / (c * ch);"),
    ("v.F term over c chat", "Cc = (S(2.0) * chiE - chiF) * vF / (c * c);",
     "Cc = (S(2.0) * chiE - chiF) * vF / (c * ch);"),
    ("R over tau c", "S Er = (A + Cc - R / (tau * ch)) / B;", "S Er = (A + Cc - R / (tau * c)) / B;"),
    ("order-1 flux denominator with c", "Fnew[k] = num / (S(1.0) + ch * chiF * tau);",
     "Fnew[k] = num / (S(1.0) + c * chiF * tau);"),
    ("momentum over c^2", "Pnew[k] = P0[k] - (Fnew[k] - F0[k]) / (c * ch);",
     "Pnew[k] = P0[k] - (Fnew[k] - F0[k]) / (c * c);"),
    ("flux rows with c^2", "phim[1 + k] = c * ch * Um[0] * Dm[d][k];",
     "phim[1 + k] = c * c * Um[0] * Dm[d][k];"),
    # stage coefficients of PD-ARS (Sec. 3.2)
    ("stage-2 source over dt", "p->scheme == 0 ? 0.5 * dt : dt, status", "p->scheme == 0 ? dt : dt, status"),
    ("stage-2 transport over dt", "if (r < nr) comb = comb + S(0.5 * dt) * s[q];",
     "if (r < nr) comb = comb + S(dt) * s[q];"),
    ("stage 2 without the average of y^n", "S comb = S(0.5) * (y[q] + yh[q]);", "S comb = yh[q];"),
    ("stage-1 source over dt/2", "apply_source(p, g, yh.data(), rho, kP, kF, kE, jS, dt, status",
     "apply_source(p, g, yh.data(), rho, kP, kF, kE, jS, 0.5 * dt, status"),
    # order-2 terms and the gas temperature
    ("emission without its order-2 factor", "S A = chiP * ar * (T2 * T2) * Afac;",
     "S A = chiP * ar * (T2 * T2);"),
    ("order-2 B: v.D.v sign",
     "B = chiE * (S(1.0) + S(0.5) * beta2) - (chiF - chiE) * (beta2 + vDv / (c * c));",
     "B = chiE * (S(1.0) + S(0.5) * beta2) - (chiF - chiE) * (beta2 - vDv / (c * c));"),
    ("order-2 flux matrix without beta^2",
     "const S a = S(1.0) + ch * chiF * (S(1.0) + S(0.5) * beta2) * tau;",
     "const S a = S(1.0) + ch * chiF * tau;"),
    ("order-2 flux matrix: (chi_F - chi_E) term sign",
     "const S bfac = ch * tau * (chiF - chiE) * S(2.0) / (c * c);",
     "const S bfac = -ch * tau * (chiF - chiE) * S(2.0) / (c * c);"),
    ("kinetic energy dropped from T", "S T = (Egas - KE) / Cv;", "S T = Egas / Cv;"),
    ("kinetic energy dropped from the converged T", "const S Tn = (Egas - KE) / Cv;",
     "const S Tn = Egas / Cv;"),
    # transport pieces
    ("HLL speed without its square root", "S smax_ = ch * ssqrt(smax(Dm[d][d], Dp[d][d]));",
     "S smax_ = ch * smax(Dm[d][d], Dp[d][d]);"),
    ("closure isotropic part sign", "S a = S(0.5) * (S(1.0) - chi);", "S a = S(0.5) * (S(1.0) + chi);"),
]


def _build(src_text, out_dir, tag):
    path = os.path.join(out_dir, f"oracle_{tag}.cpp")
    lib = os.path.join(out_dir, f"liboracle_{tag}.so")
    with open(path, "w") as f:
        f.write(src_text)
    cmd = ["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", path, "-o", lib]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return lib


def _run_pins(lib):
    env = dict(os.environ, RHD_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    return r.returncode, r.stdout[-400:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    base = open(SRC).read()
    texts = [("control", base)]
    for i, (name, old, new) in enumerate(MUTANTS):
        assert base.count(old) == 1, f"mutant {name!r}: the text must occur exactly once"
        texts.append((f"m{i}", base.replace(old, new)))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        libs = dict(zip([t for t, _ in texts],
                        ex.map(lambda tt: _build(tt[1], str(tmp_path), tt[0]), texts)))
        results = dict(zip(libs, ex.map(_run_pins, libs.values())))
    rc, out = results["control"]
    assert rc == 0, f"unmodified oracle fails its pins:\n{out}"
    survivors = [MUTANTS[int(t[1:])][0] for t, (rc, _) in results.items()
                 if t != "control" and rc == 0]
    assert not survivors, f"planted mistakes that no pin catches: {survivors}"
