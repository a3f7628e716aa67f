"""Register budget of the hot kernels (CPU: compiles the device code for gfx950
and reads the compiler's resource report).  A kernel that spills to scratch
memory runs several times slower; this guards the stencil, network and
deflation kernels and the Schwarz half-sweeps and face corrections of the
mixed-precision solver against changes that push them over the register file."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1011_0911_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, kernel-name pattern on the demangled name) that must not spill; for
# the stencil kernels the 32-bit-offset variants (every field below 4 GiB, the
# case of all workloads here)
HOT = [
    ("qdd_dirac.hip", r"k_dhat_a<[^,]+, 1, true,"),
    ("qdd_dirac.hip", r"k_dhat_b<[^,]+, 1, true,"),
    ("qdd_dirac.hip", r"k_dhat_staged<[^>]+, true>"),
    ("qdd_dirac.hip", r"k_dw<[^,]+, 1, true,"),
    ("qdd_net.hip", r"k_net_layer_mx<"),
    ("qdd_net.hip", r"k_net_wgrad_mx<"),
    ("qdd_sap.hip", r"k_sap_lds<"),
    ("qdd_sap.hip", r"k_sap_half<"),
    ("qdd_sap.hip", r"k_sap_rhs<[^,]+, [^,]+, true>"),
    ("qdd_sap.hip", r"k_sap_face<"),
    ("qdd_dfl.hip", r"k_block_orth"),
    ("qdd_dfl.hip", r"k_block_dots<"),
]


def resources(src):
    out = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops", "--offload-device-only", "-Rpass-analysis=kernel-resource-usage", "-c",
                          os.path.join(CSRC, src), "-o", os.devnull], capture_output=True, text=True, cwd=CSRC)
    assert out.returncode == 0, out.stderr[-2000:]
    rows, cur = [], None
    for line in out.stderr.splitlines():
        m = re.search(r"remark: +(Function Name|ScratchSize \[bytes/lane\]): (\S+)", line)
        if not m:
            continue
        if m.group(1) == "Function Name":
            name = subprocess.run(["c++filt", m.group(2)], capture_output=True, text=True).stdout.strip()
            cur = {"name": name}
            rows.append(cur)
        else:
            cur["scratch"] = int(m.group(2))
    return rows


SOURCES = sorted({s for s, _ in HOT})


@pytest.fixture(scope="module")
def reports():
    """The resource reports of every source, compiled side by side."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        return dict(zip(SOURCES, ex.map(resources, SOURCES)))


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("c++filt") is None, reason="needs hipcc and c++filt")
@pytest.mark.parametrize("src", SOURCES)
def test_hot_kernels_do_not_spill(reports, src):
    rows = reports[src]
    pats = [p for s, p in HOT if s == src]
    checked = 0
    for r in rows:
        if any(re.search(p, r["name"]) for p in pats):
            checked += 1
            assert r.get("scratch", 0) == 0, f"{r['name'][:120]} uses {r['scratch']} bytes of scratch per lane"
    assert checked > 0, f"no kernel of {src} matched {pats}"
