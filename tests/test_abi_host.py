"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects bad input before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hough_tf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hough_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    names = _declared()
    assert "hough_find" in names and "hough_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(hough.EXPORTS) == set(names)


def test_config_default_and_status_strings():
    from paper_2511_02742_amd import hough
    cfg = hough.default_config()
    assert (cfg.n_theta, cfg.n_rho, cfg.min_votes, cfg.peak_mode, cfg.nms_radius) == (1024, 1024, 6, 1, 1)
    assert cfg.rho_min == -500.0 and cfg.rho_max == 500.0 and cfg.n_vanes == 40
    lib = hough.load_library()
    assert lib.hough_status_string(0) == b"ok"
    assert lib.hough_status_string(-6) == b"invalid hit data"


def test_struct_layouts_match_header(tmp_path):
    """Compiles the public header with the host C compiler and compares the
    struct layouts with the Python binding's."""
    import subprocess
    from paper_2511_02742_amd import hough
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"hough_tf.h\"\n"
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(hough_config),"
        " offsetof(hough_config, min_votes), offsetof(hough_config, coarse_rho), sizeof(hough_candidate),"
        " offsetof(hough_candidate, hit_offset), offsetof(hough_candidate, rho)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(hough.HoughConfig), hough.HoughConfig.min_votes.offset,
            hough.HoughConfig.coarse_rho.offset, hough.cand_dtype.itemsize,
            hough.cand_dtype.fields["hit_offset"][1], hough.cand_dtype.fields["rho"][1]]
    assert got == want


@pytest.mark.parametrize("kw,why", [
    ({"n_theta": 0}, "n_theta"), ({"min_votes": 0}, "min_votes"), ({"peak_mode": 3}, "peak_mode"),
    ({"rho_max": -600.0}, "rho_max"), ({"wg_threads": 128}, "wg_threads"), ({"nms_radius": 17}, "nms_radius"),
    # coarse-to-fine: the factors must divide the grid (10 does not divide
    # 1024), be 0 outside mode 2, and both histograms must fit LDS
    ({"peak_mode": 2}, "coarse"), ({"coarse_theta": 10}, "coarse"),
    ({"peak_mode": 2, "n_theta": 180, "n_rho": 1000, "coarse_theta": 7}, "coarse"),
    ({"peak_mode": 2, "n_theta": 180, "n_rho": 1000, "coarse_rho": -1}, "coarse"),
    ({"peak_mode": 2, "n_theta": 180, "n_rho": 1000, "coarse_theta": 1, "coarse_rho": 1}, "16384")])
def test_create_rejects_bad_config(kw, why):
    from paper_2511_02742_amd import hough
    cfg = hough.default_config(**kw)
    lib = hough.load_library()
    h = ctypes.c_void_p()
    st = lib.hough_create(ctypes.byref(cfg), 0, ctypes.byref(h))
    assert st == hough.HOUGH_ERR_INVALID_ARG
    assert not h.value
    assert why in lib.hough_last_error(None).decode()


def test_null_and_bad_context_rejected():
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    assert lib.hough_destroy(None) == 0
    mc, mh = ctypes.c_int64(), ctypes.c_int64()
    assert lib.hough_output_bounds(None, 1, 10, ctypes.byref(mc), ctypes.byref(mh)) == hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_find(None, None, 1, 0, None, None, None, None, 0, None, 0, None) == \
        hough.HOUGH_ERR_INVALID_ARG


def test_server_struct_layouts_match_header(tmp_path):
    import subprocess
    from paper_2511_02742_amd import hough
    src = tmp_path / "slayout.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"hough_tf.h\"\n"
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(hough_server_config),"
        " offsetof(hough_server_config, max_batch_hits), offsetof(hough_server_config, queue_events),"
        " sizeof(hough_served), offsetof(hough_served, cand_offset), offsetof(hough_served, t_done),"
        " sizeof(hough_server_stats), offsetof(hough_server_stats, device_bytes),"
        " offsetof(hough_server_stats, results_waiting), offsetof(hough_server_config, device_bytes),"
        " offsetof(hough_server_stats, max_device_bytes_in_use)); return 0;}\n")
    exe = tmp_path / "slayout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    sd = hough.served_dtype
    want = [ctypes.sizeof(hough.ServerConfig), hough.ServerConfig.max_batch_hits.offset,
            hough.ServerConfig.queue_events.offset, sd.itemsize, sd.fields["cand_offset"][1],
            sd.fields["t_done"][1], 16 * 8, 8 * hough.SERVER_STAT_NAMES.index("device_bytes"),
            8 * hough.SERVER_STAT_NAMES.index("results_waiting"), hough.ServerConfig.device_bytes.offset,
            8 * hough.SERVER_STAT_NAMES.index("max_device_bytes_in_use")]
    assert got == want


def test_server_rejects_bad_arguments_without_a_device():
    """Argument checks that return before any device work."""
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    cfg = hough.default_config()
    h = ctypes.c_void_p()
    bad = hough.ServerConfig()
    bad.lanes = 9
    assert lib.hough_server_create(ctypes.byref(cfg), 0, ctypes.byref(bad), ctypes.byref(h)) == \
        hough.HOUGH_ERR_INVALID_ARG
    bad = hough.ServerConfig()
    bad.reserved = 1
    assert lib.hough_server_create(ctypes.byref(cfg), 0, ctypes.byref(bad), ctypes.byref(h)) == \
        hough.HOUGH_ERR_INVALID_ARG
    bad = hough.ServerConfig()
    bad.device_bytes = -1
    assert lib.hough_server_create(ctypes.byref(cfg), 0, ctypes.byref(bad), ctypes.byref(h)) == \
        hough.HOUGH_ERR_INVALID_ARG
    assert not h.value
    assert lib.hough_server_destroy(None) == 0
    n = ctypes.c_int32()
    assert lib.hough_server_submit(None, 0, None, None, None, None, None, ctypes.byref(n)) == \
        hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_server_poll(None, 0, None, None, 0, None, 0, ctypes.byref(n)) == hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_server_drain(None, 0.0) == hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_server_clock(None) == -1.0


def _device_build(extra):
    import shutil
    import subprocess
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_2511_02742_amd import build
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-I", os.path.join(ROOT, "include"),
           "-I", build.CSRC, os.path.join(build.CSRC, "hough_kernels.hip")] + extra
    return subprocess.run(cmd, capture_output=True, text=True)


def test_kernels_keep_scratch_out_of_their_loops(tmp_path):
    """The finder, sweep and band kernels keep their working set in registers
    and LDS: no scratch at all (the finders run at 128 VGPRs at every width,
    so that smaller workgroups can share a CU; addresses derived from the
    thread index are computed where used, not held across the kernel). Were
    a spill to come back, it must stay out of the per-row vote, recount and
    association loops (a spill there once cost a quarter of the kernel's
    speed). Compiles the device code for gfx950 and reads the resource
    remarks and the assembly."""
    out = _device_build(["-c", "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]).stderr
    blocks = re.split(r"remark: Function Name: ", out)[1:]
    seen = 0
    for blk in blocks:
        name = blk.split()[0]
        if "k_find" not in name and "k_sweep" not in name and "k_band" not in name:
            continue
        seen += 1
        scratch = int(re.search(r"ScratchSize \[bytes/lane\]: (\d+)", blk).group(1))
        assert scratch == 0, (name, scratch)
    assert seen >= 7
    asm = tmp_path / "k.s"
    r = _device_build(["-S", "-o", str(asm)])
    assert r.returncode == 0, r.stderr[-2000:]
    text = asm.read_text()
    kernels = 0
    for m in re.finditer(r"^(_Z\S*k_find\S*):", text, re.M):
        kernels += 1
        body = text[m.end():text.index(".Lfunc_end", m.end())]
        depth = deepest = 0
        for line in body.splitlines():
            if re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):", line):
                d = re.findall(r"Depth=(\d+)", line)
                depth = max(int(x) for x in d) if d else 0
                deepest = max(deepest, depth)
            elif "scratch_" in line:
                assert depth <= 1, (m.group(1), line.strip(), depth)
        assert deepest >= 3, (m.group(1), deepest)   # the vote loops were seen
    assert kernels == 3


def test_refit_calls_reject_bad_arguments_without_a_device():
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    E = hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_refit_init(None, -1, None, None, None, None, 40, None, None, None, None) == E
    assert lib.hough_refit_init(None, 1, None, None, None, None, 40, None, None, None, None) == E
    assert lib.hough_refit_chi2(None, 0, None, None, None, None, 40, None, None, None, 0.0, None) == E
    assert lib.hough_refit_grad(None, 2, None, None, None, None, 0, None, None, None, None, 0.055, None) == E
    assert lib.hough_refit_gauss_newton(None, 0, None, None, None, None, 40, None, None, None, None, -1, 1e-3,
                                        0.055, None) == E
    assert lib.hough_refit_gather(None, 1, None, None, None, None, None, None, None, None, None, None) == E
    # nothing to do is not an error
    assert lib.hough_refit_chi2(None, 0, None, None, None, None, 40, None, None, None, 0.055, None) == 0


def test_lds_peak_rejects_bad_arguments_without_a_device():
    import ctypes as C
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    out = C.c_double()
    assert lib.hough_lds_peak(0, None, 2, C.byref(out)) == hough.HOUGH_ERR_INVALID_ARG
    assert lib.hough_lds_peak(0, None, 0, None) == hough.HOUGH_ERR_INVALID_ARG


def test_tw_struct_layouts_and_defaults(tmp_path):
    import subprocess
    from paper_2511_02742_amd import hough
    src = tmp_path / "tw.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"hough_tf.h\"\n"
        "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(hough_tw_config),"
        " offsetof(hough_tw_config, max_track_hits), sizeof(hough_track), offsetof(hough_track, hit_offset),"
        " offsetof(hough_track, carried)); return 0;}\n")
    exe = tmp_path / "tw"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(hough.TwConfig), hough.TwConfig.max_track_hits.offset, hough.track_dtype.itemsize,
                   hough.track_dtype.fields["hit_offset"][1], hough.track_dtype.fields["carried"][1]]
    tw = hough.tw_config()
    assert (tw.window_ns, tw.step_ns, tw.gate_r_mm, tw.gate_z_mm, tw.gate_t_ns, tw.max_track_hits) == \
        (10.0, 5.0, 10.0, 4.0, 2.0, 64)


def test_tw_find_rejects_bad_arguments_without_a_device():
    from paper_2511_02742_amd import hough
    lib = hough.load_library()
    tw = hough.tw_config()
    # a bad context is refused before anything else
    assert lib.hough_tw_find(None, None, ctypes.byref(tw), 1, 0, ctypes.c_void_p(8), None, None, None, None, 1,
                             None, 0, None, 0, ctypes.c_void_p(8)) == hough.HOUGH_ERR_INVALID_ARG
