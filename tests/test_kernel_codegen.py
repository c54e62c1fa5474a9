"""Code-generation checks of the blind-rotation kernels for gfx950 (CPU only:
hipcc cross-compiles).  They guard properties the throughput depends on and
that a harmless-looking source change can lose without any parity test
noticing:
  * the N = 1024 kernels, the default N = 2048 one and the one-limb N = 2048
    ones fit two waves per SIMD without scratch;
  * no buffer load of the key or the transform tables sits in a waterfall
    loop (a descriptor the compiler cannot prove uniform is re-read lane by
    lane around every load: readfirstlane + 64-bit compare + exec loop)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_09025_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")


@pytest.fixture(scope="module")
def compiled(tmp_path_factory):
    from paper_2309_09025_amd import build as B
    out = tmp_path_factory.mktemp("codegen")
    asm = str(out / "pbs.s")
    flags = [f for f in B.FLAGS if f not in ("-fPIC",)]
    r = subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", "-x", "hip",
                        "-Rpass-analysis=kernel-resource-usage",
                        os.path.join(CSRC, "pbs.hip"), "-o", asm],
                       capture_output=True, text=True, check=True)
    usage = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if name and m:
            usage[name][m.group(1).strip()] = int(m.group(2))
    with open(asm) as fh:
        text = fh.read()
    return usage, text


def _br(usage, args, held=False, heldi=0):
    """Resource record of blind_rotate_kernel<args..., held, heldi>."""
    mangled = ("_ZN2fs19blind_rotate_kernelI" + "".join(f"Li{a}E" for a in args)
               + f"Lb{int(held)}ELi{heldi}E" + "EEvNS_6BrArgsE")
    assert mangled in usage, sorted(k for k in usage if "blind_rotate" in k)
    return mangled, usage[mangled]


@pytest.mark.parametrize("args", [(10, 3, 7, 1, 0, 2, 1, 1), (10, 3, 7, 1, 1, 2, 1, 1),
                                  (10, 3, 7, 1, 2, 2, 1, 1), (11, 2, 10, 2, 3, 2, 1, 1),
                                  (11, 2, 10, 1, 2, 2, 1, 1), (11, 2, 10, 1, 1, 2, 2, 1),
                                  (10, 3, 7, 1, 2, 1, 1, 8), (10, 3, 7, 1, 0, 2, 1, 8)])
def test_two_wave_kernels_have_no_scratch(compiled, args):
    usage, _ = compiled
    _, u = _br(usage, args)
    assert u.get("ScratchSize", 0) == 0, u
    assert u.get("Occupancy", 0) >= 2, u


@pytest.mark.parametrize("args,heldi", [((10, 3, 7, 1, 0, 2, 1, 1), 0), ((10, 3, 7, 1, 3, 2, 1, 1), 0),
                                        ((10, 3, 7, 1, 1, 2, 1, 1), 0), ((11, 2, 10, 1, 3, 2, 1, 1), 1),
                                        ((11, 2, 10, 1, 0, 2, 1, 1), 1), ((11, 2, 10, 1, 1, 2, 1, 1), 0),
                                        ((11, 2, 10, 1, 0, 2, 1, 2), 1)])
def test_held_root_kernels_fit_two_waves_without_scratch(compiled, args, heldi):
    """The variants holding the forward transforms' roots in registers for
    the whole job (and, for the one-limb key, the inverse transforms' round-B'
    roots)."""
    usage, _ = compiled
    _, u = _br(usage, args, held=True, heldi=heldi)
    assert u.get("ScratchSize", 0) == 0, u
    assert u.get("Occupancy", 0) >= 2, u


def test_small_batch_forms_have_no_scratch(compiled):
    """N = 1024 two-group kernels: the split form (held forward roots, two
    waves per SIMD when three jobs share a CU) and the paired form (one wave
    per SIMD, every root held) run without scratch."""
    usage, _ = compiled
    _, u = _br(usage, (10, 3, 7, 1, 1, 2, 2, 1), held=True)
    assert u.get("ScratchSize", 0) == 0 and u.get("Occupancy", 0) >= 2, u
    _, u = _br(usage, (10, 3, 7, 1, 1, 1, 2, 2), held=True, heldi=2)
    assert u.get("ScratchSize", 0) == 0 and u.get("Occupancy", 0) >= 1, u


def test_held_inverse_root_kernel_fits_two_waves_without_scratch(compiled):
    """The N = 1024 variant holding both the forward and the inverse
    transforms' per-thread roots for the whole job."""
    usage, _ = compiled
    _, u = _br(usage, (10, 3, 7, 1, 0, 2, 1, 1), held=True, heldi=2)
    assert u.get("ScratchSize", 0) == 0, u
    assert u.get("Occupancy", 0) >= 2, u


def test_no_waterfall_loops_in_blind_rotation(compiled):
    usage, text = compiled
    for name in (k for k in usage if "blind_rotate" in k and "kernel" in k):
        body = text.split(f"\n{name}:", 1)[1].split("s_endpgm", 1)[0]
        # a waterfall loop compares a readfirstlane'd 64-bit value with the
        # vector register it came from
        assert "v_cmp_eq_u64" not in body, name


@pytest.mark.parametrize("name", ["_ZN2fs24blind_rotate_rows_kernelILi11ELi2ELi10ELi2EEEvNS_6BrArgsE",
                                  "_ZN2fs27blind_rotate_halfrow_kernelILi3ELi7EEEvNS_6BrArgsE"])
def test_row_kernels_use_lds_float_atomics(compiled, name):
    """The latency kernels (one group per digit row at N = 2048, one wave per
    digit row half at N = 1024) sum the rows' products with hardware LDS
    binary64 atomic adds (a compare-and-swap loop would serialise them), and
    use no scratch."""
    usage, text = compiled
    assert name in usage, sorted(k for k in usage if "row" in k)
    assert usage[name].get("ScratchSize", 0) == 0
    body = text.split(f"\n{name}:", 1)[1].split("s_endpgm", 1)[0]
    assert "ds_add_f64" in body or "ds_add_rtn_f64" in body
    assert "ds_cmpst" not in body and "ds_cmpswap" not in body


def test_half_row_kernel_fits_its_twelve_waves(compiled):
    """12 waves per job, three per SIMD: at most 168 registers."""
    usage, _ = compiled
    u = usage["_ZN2fs27blind_rotate_halfrow_kernelILi3ELi7EEEvNS_6BrArgsE"]
    assert u.get("VGPRs", 0) + u.get("AGPRs", 0) <= 168, u


def test_tuned_two_limb_lockstep_kernel_spills_only_outside_its_loop(compiled):
    """The tuned N = 2048 two-limb kernel (two jobs per workgroup in
    lockstep) sits at 256 registers with one value spilled: allowed only as
    one store and one reload in the whole kernel (prologue and extraction
    epilogue), never a spill inside the CMux loop."""
    usage, text = compiled
    name, u = _br(usage, (11, 2, 10, 2, 3, 2, 1, 2))
    assert u.get("Occupancy", 0) >= 2, u
    assert u.get("ScratchSize", 0) <= 8, u
    body = text[text.index(name + ":"):]
    body = body[:body.index("s_endpgm")]
    assert len(re.findall(r"scratch_(load|store)", body)) <= 2
