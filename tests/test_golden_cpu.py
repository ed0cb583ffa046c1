"""Values the paper prints (tests/golden/paper_constants.txt, each with its
section) against the benchmark's definitions: the Flop count of one
interaction of Eq. 1 under the paper's counting, the fiducial accuracy
parameter and particle counts, and the printed rate against the printed peak."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _constants():
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, value, section, _ = (t.strip() for t in line.split("|", 3))
            assert section.startswith("Sec."), name
            out[name] = float(value)
    return out


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_flops_per_interaction_follow_the_papers_counting():
    c = _constants()
    b = _bench()
    # Eq. 1 per interaction: three subtractions for the separation, three FMAs
    # for r^2 + eps^2, the reciprocal square root, three multiplications
    # (m r^-1, r^-2, their product) and three FMAs into the sum. An FMA counts
    # as a multiply and an add (our reading: the paper names the profiler's
    # FMA metric without restating its convention); the reciprocal square
    # root counts as the paper prints.
    fma = 2
    flops = 3 * 1 + 3 * fma + c["rsqrt_flops"] + 3 * 1 + 3 * fma
    assert flops == b.FLOP_PER_INTERACTION == 22


def test_bench_defaults_are_the_papers_fiducial_configuration():
    c = _constants()
    args = _bench().build_parser().parse_args([])
    assert args.delta == c["delta_acc"] == 2.0 ** -9
    assert args.n == c["n_fiducial"] == 2 ** 23
    assert c["n_largest"] == 25 * 2 ** 20


def test_printed_rate_and_peak_agree():
    c = _constants()
    frac = c["sustained_tflops_n_largest"] / c["v100_fp32_peak_tflops"]
    assert abs(frac - c["sustained_fraction_n_largest"]) < 0.005
