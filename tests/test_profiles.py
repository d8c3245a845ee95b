"""The committed rocprofv3 counter summaries and the kernel source: bench.py
reads their HBM traffic and busy fractions only while the recorded SHA-256
matches the source (else it reports null); a summary of an older source is
skipped here as stale, and every current one is checked for consistency."""
import hashlib
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2310_03979_amd", "csrc", "srm3_kernels.hip")
SUMMARIES = ["pairsum_mfma_c1_256x1024_b64_counters.md", "pairsum_mfma_c2_512x8192_w2048_b16_counters.md",
             "pairsum_c1_256x1024_b64_counters.md", "pairsum_c2_512x8192_w2048_b16_counters.md"]


def _field(path, key):
    for line in open(path):
        if line.startswith("- " + key + ": "):
            return line.split(": ", 1)[1].strip().strip("`")
    return None


def _current(name):
    path = os.path.join(ROOT, "profiles", name)
    digest = hashlib.sha256(open(SRC, "rb").read()).hexdigest()
    return os.path.exists(path) and _field(path, "kernel source sha256") == digest


@pytest.mark.parametrize("name", SUMMARIES)
def test_counter_summary_matches_kernel_source(name):
    import bench
    import srm3_inputs as inp
    wl = inp.C1 if "_c1_" in name else inp.C2
    kernel = "mfma" if name.startswith("pairsum_mfma") else "vector"
    if not _current(name):
        assert bench.counter_traffic(wl, kernel) is None
        pytest.skip(f"{name} predates the kernel source (bench.py reports its traffic as null)")
    assert float(_field(os.path.join(ROOT, "profiles", name), "HBM bytes per launch")) > 0
    assert bench.counter_traffic(wl, kernel) > 0


def test_bench_reads_the_summaries():
    import bench
    import srm3_inputs as inp
    if not all(_current(n) for n in SUMMARIES[:1] + SUMMARIES[2:3]):
        pytest.skip("c1 summaries predate the kernel source")
    assert bench.counter_traffic(inp.C1, "mfma") > 0
    assert 0.5 < bench.counter_valu(inp.C1, "mfma", "* MFMA busy") <= 1.0
    assert 0.5 < bench.counter_valu(inp.C1, "vector") <= 1.0


def test_mfma_instruction_model_matches_the_counters():
    """The host count of the matrix-core kernel's MFMAs (reported by bench.py)
    equals SQ_INSTS_MFMA of the profiled launches, and the useful share of the
    issued products (pair terms over 1024 products per three MFMAs) is the
    figure quoted for the kernel."""
    import bench
    import srm3_inputs as inp
    if not all(_current(n) for n in SUMMARIES[:2]):
        pytest.skip("matrix-core summaries predate the kernel source")
    for wl, name in ((inp.C1, "pairsum_mfma_c1_256x1024_b64_counters.md"),
                     (inp.C2, "pairsum_mfma_c2_512x8192_w2048_b16_counters.md")):
        measured = None
        for line in open(os.path.join(ROOT, "profiles", name)):
            if line.startswith("| SQ_INSTS_MFMA |"):
                measured = float(line.split("|")[2])
        assert measured is not None
        model = bench.mfma_instructions(wl) * wl.batch
        assert abs(model - measured) <= 1e-4 * measured, (name, model, measured)
    useful = bench.pair_terms_total(inp.C1) / (bench.mfma_instructions(inp.C1) / 3 * 1024)
    assert 0.93 < useful < 0.94


@pytest.mark.parametrize("name", SUMMARIES)
def test_counter_summary_duration_is_its_kernels(name):
    """The duration a counter summary derives its rates from is the kernel
    trace's average for the same kernel (full name, template arguments
    included) in the same workload, and the clock it implies is the chip's."""
    import re
    path = os.path.join(ROOT, "profiles", name)
    if not _current(name):
        pytest.skip(f"{name} predates the kernel source")
    text = open(path).read()
    m = re.search(r"kernel duration ([0-9.]+) ms: .*? of `([^`]+)`", text)
    assert m, name
    ms, kernel = float(m.group(1)), m.group(2)
    wl = name.split("_counters")[0].split("pairsum_mfma_")[-1].split("pairsum_")[-1]
    trace = os.path.join(ROOT, "profiles", f"pairsum_{wl}_kernel_trace.md")
    avgs = []
    for line in open(trace):
        cells = [c.strip() for c in line.split("|")]
        if len(cells) > 6 and cells[1] == f"`{kernel}`":
            avgs.append(float(cells[5]))
    assert any(abs(a - ms) <= 5e-4 * ms for a in avgs), (name, ms, avgs)
    ghz = float(re.search(r"-> ([0-9.]+) GHz", text).group(1))
    assert 2.0 <= ghz <= 2.5, (name, ghz)


@pytest.mark.parametrize("wl", ["c1_256x1024_b64", "c2_512x8192_w2048_b16"])
def test_transform_summaries(wl):
    """Phases and transforms: one row per launch kind, measured HBM traffic
    within a small factor of the algorithmic bytes (no wasted re-reads)."""
    path = os.path.join(ROOT, "profiles", f"transforms_{wl}_counters.md")
    digest = hashlib.sha256(open(SRC, "rb").read()).hexdigest()
    if _field(path, "kernel source sha256") != digest:
        pytest.skip("transform summary predates the kernel source")
    rows = [l for l in open(path) if l.startswith("| ") and "`" in l]
    assert len(rows) == 5
    for r in rows:
        cells = [c.strip() for c in r.split("|")]
        ratio = float(cells[8])
        assert 0.9 < ratio < 2.5, r
