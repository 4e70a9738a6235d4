"""Mutation check of the oracle's pins: plant one plausible mistake at a time
in a private copy of the oracle's C source (a dropped term, a wrong sign or
index, a swapped operand, a wrong constant), rebuild that copy and run the
oracle pin tests against it.  Every planted mistake must make at least one
pin fail.  CPU only; nothing here touches the oracle in the repository."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what the mistake is, original text, mutated text)
MUTATIONS = [
    ("half kick doubled", "const double hk = 0.5 * ms;", "const double hk = ms;"),
    ("rotation sign in z", "double qz = mz + (px * sy - py * sx);", "double qz = mz + (px * sy + py * sx);"),
    ("cross product operand order", "double pz = mz + (mx * ty - my * tx);",
     "double pz = mz + (my * tx - mx * ty);"),
    ("deposit to the wrong node", "S[j + 1] += w1;", "S[j] += w1;"),
    ("gradient sign", "E[j] = (phi[j - 1] - phi[j + 1]) / (2.0 * dx);",
     "E[j] = (phi[j + 1] - phi[j - 1]) / (2.0 * dx);"),
    ("wall closure term dropped", "E[0] = -(phi[1] - phi[0]) / dx - rho[0] * dx / (2.0 * c->eps0);",
     "E[0] = -(phi[1] - phi[0]) / dx;"),
    ("elastic mass ratios swapped", "P->vx[p] = am * vx + bm * g * d[0];",
     "P->vx[p] = bm * vx + am * g * d[0];"),
    ("ionisation energy not split", "const double e2 = e_tot - e1;", "const double e2 = e_tot;"),
    ("Philox key constant", "k0 += 0x9E3779B9u;", "k0 += 0x9E3779B8u;"),
    ("ionisation threshold ignored", "} else if (v2 >= v2_iz) {", "} else if (1) {"),
    ("source counts one wall", "const int64_t n_pairs = s->cnt.absorbed[ki][0] + s->cnt.absorbed[ki][1];",
     "const int64_t n_pairs = s->cnt.absorbed[ki][0];"),
    ("events not ranked by parent id", "if (n_ev > 1) qsort", "if (0) qsort"),
    ("isotropic cosine range", "double cc = 1.0 - 2.0 * u01(a);", "double cc = 1.0 - u01(a);"),
    ("periodic background dropped", "rho[j] = acc / V + rho_bg;", "rho[j] = acc / V;"),
    ("Poisson pivot off by one", "const double den = -(u + 1.0) / u;",
     "const double den = -(u + 2.0) / u;"),
    ("Boris uses dt, not dt/2",
     "const double tm = (c->q[k] / c->m[k]) * c->B0 * (0.5 * (c->dt * (double)sub_of(c, k)));",
     "const double tm = (c->q[k] / c->m[k]) * c->B0 * (c->dt * (double)sub_of(c, k));"),
    ("subcycled advance ignores nstep", "x[p] = x[p] + ms * vx[p];", "x[p] = x[p] + vx[p];"),
    ("subcycled collision test uses one step", "double P = -expm1(-(nu_max * (double)sub_of(c, k)));",
     "double P = -expm1(-nu_max);"),
    ("atoms consumed largest key first", "if (p->key != q->key) return (p->key > q->key) - (p->key < q->key);",
     "if (p->key != q->key) return (p->key < q->key) - (p->key > q->key);"),
    ("ion left at the parent, not the atom", "if (ev[r].target >= 0) ev[r].x = N->x[ev[r].target];",
     "if (0) ev[r].x = N->x[ev[r].target];"),
    ("excitation loses no energy", "const double g = sqrt(v2 - v2_ex);", "const double g = sqrt(v2);"),
    ("constant rate taken at |v|", "const double rr = r - ((nl * c->sig_iz) * dx) * vcap_hat;",
     "const double rr = r - ((nl * c->sig_iz) * dx) * sqrt(v2);"),
    ("neutral density without the node volume", "n = (c->w[kn] * ((double)Sj * two_m32)) / V;",
     "n = (c->w[kn] * ((double)Sj * two_m32)) / dx;"),
    ("mean instead of local neutral density", "nl = neutral_density_at(s, P->x[p]);",
     "nl = 0.5 * (s->nn[0] + s->nn[c->nc / 2]);"),
    ("field left on without the solver", "    if (c->field_off) {", "    if (0) {"),
    ("new electrons not counted in n_e", "append(s, ke, xe[r], ev[r].ve, s->cnt.next_id + 2 * (uint64_t)r);",
     "(void)xe;"),
    ("kinetic energy without the half", "out->ke[k] = 0.5 * c->m[k] * c->w[k] * (vs * vs) * s2;",
     "out->ke[k] = c->m[k] * c->w[k] * (vs * vs) * s2;"),
    ("kinetic energy with dx/dt not squared", "c->w[k] * (vs * vs) * s2;", "c->w[k] * vs * s2;"),
    ("momentum z from vx", "pz += P->vz[p];", "pz += P->vx[p];"),
    ("field energy with full wall-node volumes", "fe += s->E[j] * s->E[j] * V;",
     "fe += s->E[j] * s->E[j] * c->dx;"),
    ("periodic field energy counts node nc twice", "for (int32_t j = 0; j < nc; ++j) fe +=",
     "for (int32_t j = 0; j <= nc; ++j) fe +="),
    ("field energy without the half", "out->field_energy = 0.5 * c->eps0 * fe;",
     "out->field_energy = c->eps0 * fe;"),
    ("FP32 form leaves the last cell", "if (cell + 1.0 < (double)nc) {", "if (1) {"),
    ("FP32 form keeps an offset of one", "if (f >= 1.0f) {", "if (f > 1.0f) {"),
    ("x = nc kept", "if (x >= L) { s->cnt.absorbed[k][1]++; continue; }",
     "if (x > L) { s->cnt.absorbed[k][1]++; continue; }"),
    ("x = 0 absorbed", "if (x < 0.0) { s->cnt.absorbed[k][0]++; continue; }",
     "if (x <= 0.0) { s->cnt.absorbed[k][0]++; continue; }"),
]


def _pin_tests():
    here = os.path.join(ROOT, "tests")
    return sorted(f for f in os.listdir(here)
                  if f.startswith("test_oracle_") and f.endswith(".py")
                  and f != os.path.basename(__file__))


def _run(mut):
    name, a, b = mut
    with tempfile.TemporaryDirectory(prefix="orc_mut_") as tmp:
        shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tmp, "oracle"),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
        shutil.copytree(os.path.join(ROOT, "pic_inputs"), os.path.join(tmp, "pic_inputs"),
                        ignore=shutil.ignore_patterns("__pycache__"))
        tdir = os.path.join(tmp, "tests")
        os.makedirs(tdir)
        for f in _pin_tests() + ["conftest.py", "rocrand_philox_kat.cpp"]:
            shutil.copy(os.path.join(ROOT, "tests", f), tdir)
        shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(tdir, "golden"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp)
        src = os.path.join(tmp, "oracle", "pic_oracle.c")
        with open(src) as f:
            s = f.read()
        if a not in s:
            return name, "not applied"
        with open(src, "w") as f:
            f.write(s.replace(a, b))
        env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu",
                            "-p", "no:cacheprovider"], cwd=tmp, env=env, capture_output=True,
                           text=True, timeout=900)
        return name, ("caught" if r.returncode != 0 else "survived")


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        res = list(ex.map(_run, MUTATIONS))
    bad = [(n, r) for n, r in res if r != "caught"]
    assert not bad, bad
