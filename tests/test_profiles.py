"""The committed rocprofv3 summaries belong to the committed kernels: the
traffic figures `bench.py` reports as `roofline.traffic` are read only when
`profiles/pmc_traffic.json` was taken with the current kernel source, and the
kernel profiles name that source and the command that made them."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_traffic_file_matches_the_kernel_source():
    with open(os.path.join(PROFILES, "pmc_traffic.json")) as fh:
        t = json.load(fh)
    assert t["kernel_sha"] == bench.kernel_sha()
    for name, bpc in (("D3Q13", 104), ("D3Q21", 168), ("D3V27", 216), ("D3Q27", 216)):
        b = bench.traffic_for(name, 128)
        alg = bpc * 128 ** 3
        assert t["kernels"]["%s_128" % name]["algorithmic_bytes"] == alg
        # at least the state read and written once, and not wildly above it
        assert alg <= b <= 2 * alg, (name, b, alg)


def test_kernel_profiles_name_their_source_and_command():
    sha = bench.kernel_sha()
    for f in ("sl_kernel_tgv3d_128_fp32.md", "sl_kernel_ctgv_256_d3q45.md", "sl_kernel_glc_tgv3d_128_fp32.md",
              "sl_kernel_svi_512_2048.md", "sl_kernel_adjoint_d3q27_64_fp32.md"):
        with open(os.path.join(PROFILES, f)) as fh:
            txt = fh.read()
        assert "rocprofv3 --kernel-trace --stats" in txt, f
        assert sha in txt, f
