"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a workload through every part of it (all sixteen channels, pairing
with short cells, loading from profiles, the O2(a) solver, moments, the event
log) runs in a child process with the sanitizer runtime and must finish with no
report.  CPU only."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

WORKLOAD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    from oracle import pyoracle as po
    from paper_0705_0497_amd import inputs as I
    po.LIB_PATH = {lib!r}
    procs = I.make_processes_full()
    for k, p in enumerate(procs):                 # frequent electron-ion and ion-ion events
        if p.kind in ("recomb", "edetach"):
            procs[k] = I.Process(p.name, 0, p.kind, p.target, p.e_th, p.target_mass,
                                 I.power_law_table(3e-14, 0.0, 0.5, p.e_th), {{}})
        if p.kind == "neutralize":
            p.sigma = p.sigma * 3e4
    d = I.config(1, n_total=4000, diag_every=5)
    o = po.Oracle(d, d.species(), procs)
    o.load_uniform()
    o.prepare(True)
    o.log_events(True)
    ka1 = [p.name for p in procs].index("e-a1")
    o.metastable_config(ka1, 0.1, 20.0, 0.05)
    o.step(60)
    o.metastable_update()
    o.step(30)
    m = o.moments()
    assert m["nacc"] == 90 and o.events().shape[1] == 6
    c = o.counters()
    assert c[po.C_PAIRED] > 0 and c[po.C_PAIRED_NEG] + c[po.C_DEFICIT_NEG] > 0
    x = np.linspace(0.0, 1.0, 9)
    dens = np.stack([np.full(9, 3e14), np.full(9, 6e14), np.full(9, 3e14)])
    mean = np.stack([np.full(9, 2.0), np.full(9, 0.04), np.full(9, 0.04)])
    o2 = po.Oracle(d, d.species(), procs)
    o2.load_profile(x, dens, mean)
    o2.prepare(True)
    o2.step(20)
    print("sanitized oracle ok", flush=True)
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from oracle import pyoracle as po
    lib = str(tmp_path / "liboracle_san.so")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", *po.SOURCES,
                           "-o", lib, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime for gcc here")
    env = dict(os.environ, LD_PRELOAD=" ".join(p for p in (asan, ubsan) if os.path.isabs(p)),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    script = tmp_path / "workload.py"
    script.write_text(WORKLOAD.format(root=ROOT, lib=lib))
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
