"""Memory and undefined-behaviour checks of the CPU code (no GPU needed).

* The C oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc), runs every model, the given-ancestor and sampled-slot steps, the
  searches, resampling schemes and samplers at small sizes in a child
  process; any report aborts it.
* The host runtime of the library (configuration checks, workspace layout,
  argument validation, error and clean-up paths of the C-ABI), built with
  both sanitizers by g++ against the HIP headers, with the device launches
  replaced by stand-ins that report "no device", is driven through its
  entry points the same way.  (Device code is not sanitized: GPU
  sanitizers are not available here.)"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1212_1639_amd", "csrc")


def _runtime_libs():
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True,
                           text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{name} not available")
        libs.append(p)
    return libs


def _run_sanitized(script, tmp_path):
    env = dict(os.environ, LD_PRELOAD=":".join(_runtime_libs()),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT)
    path = tmp_path / "drive.py"
    path.write_text(textwrap.dedent(script))
    r = subprocess.run([sys.executable, str(path)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=str(tmp_path))
    assert r.returncode == 0 and "ALL DONE" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", *SAN, "-o", str(lib),
                    os.path.join(ROOT, "oracle", "pf_oracle.c"), "-lm"], check=True)
    _run_sanitized(f"""
        import numpy as np
        import oracle
        oracle.build = lambda force=False: {str(lib)!r}
        from tests import _cases as C
        for model in ("ll_pf", "ll_pl", "sv_pf", "sv_pl"):
            for scheme in ("multinomial", "stratified", "systematic", "sorted_multinomial"):
                for fp32 in (False, True):
                    cfg = C.oracle_config(oracle, model, 257, 3, scheme, fp32)
                    y = C.data(model, 6)
                    r = oracle.run(cfg, y, dump=True)
                    st = r["state"][2]
                    g = oracle.run(cfg, y[3:], dump=True, state0=st, t0=3, y_prev=y[2],
                                   anc_first=r["anc"][3])
                    assert np.array_equal(g["anc"], r["anc"][3:])
                    oracle.step_slots(cfg, st, 3, y[2], y[3], np.array([0, 5, 256]))
        q, M, S = oracle.cdf(np.log(np.random.default_rng(0).random(1000)))
        u = np.random.default_rng(1).random(500)
        for m in (oracle.SEARCH_BINARY, oracle.SEARCH_CUTPOINT, oracle.SEARCH_BRUTE):
            oracle.search(q, u, m)
        L, I = oracle.cutpoint_table(q)
        oracle.cutpoint_draw(q, I, 0.3)
        for s in range(4):
            oracle.uniforms(s, 7, 2, 300)
        oracle.philox([1, 2, 3, 4], [5, 6])
        oracle.gamma_mt(3.5, 0.1, 0.4, seed=1, j=2, t=3, g=0)
        cfg = oracle.make_config(oracle.SV_PL, 1, 0, prior_mean=[0.0, 0.9],
                                 prior_prec=[1.0, 0.2, 3.0], a_s=3.0, d_s=0.5)
        post = oracle.sv_posterior(cfg, [10, 1.0, 4.0, 2.0, 1.5, 3.0])
        oracle.sv_theta(post, 0.3, 0.6, -0.2, 1.1, seed=9, j=1, t=1)
        print("ALL DONE")
    """, tmp_path)


STUBS = r'''
#include <hip/hip_runtime.h>
#include "pf_internal.h"
// device launches replaced by stand-ins that report "no device"
namespace pf {
hipError_t launch_step(int, bool, int, const StepArgs&, int, hipStream_t, bool) { return hipErrorNoDevice; }
hipError_t launch_scan_tiles(double*, int32_t, int64_t, int32_t, TileAB*, int32_t*, Totals*, DevState*, double*, const TileAB*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_spacings(int, uint64_t, uint32_t, int64_t, int32_t, double*, TileAB*, Totals*, double*, hipStream_t) { return hipErrorNoDevice; }
int32_t scan_chunks(int32_t num_tiles) { return (num_tiles + 1023) / 1024; }
hipError_t static_scratch(int32_t**) { return hipErrorNoDevice; }
hipError_t launch_fill_i32(int32_t*, int64_t, int32_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_cut_table(bool, const void*, const TileAB*, int64_t, int32_t, int32_t, int32_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch(int, bool, int, const StepArgs*, const int2*, int32_t, BatchState*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_map(const int32_t*, int32_t, int2*, hipStream_t) { return hipErrorNoDevice; }
int batch_grid(int, bool, int) { return 1; }
hipError_t launch_moments(int, const double*, int32_t, int64_t, int32_t, uint32_t, const ModelParams&, DevState*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_search(int, const double*, int64_t, const double*, int64_t, int32_t*, int32_t*, int32_t*, hipStream_t) { return hipErrorNoDevice; }
}  // namespace pf
'''


def test_host_runtime_under_sanitizers(tmp_path):
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not available")
    (tmp_path / "stubs.cpp").write_text(STUBS)
    lib = tmp_path / "libpf_san.so"
    r = subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                        *SAN, "-o", str(lib), os.path.join(CSRC, "pf_api.cpp"),
                        os.path.join(CSRC, "pf_tune.cpp"), str(tmp_path / "stubs.cpp"),
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    _run_sanitized(f"""
        import ctypes
        import numpy as np
        from paper_1212_1639_amd import pf
        pf.LIB_PATH = {str(lib)!r}
        L = pf.lib()
        vp = ctypes.c_void_p
        assert [L.pf_fields(m) for m in range(5)] == [1, 5, 1, 6, 0]
        svp = dict(x0_mean=-1.0, x0_var=0.1, prior_mean=[-0.05, 0.95], prior_prec=[1.0, 0.0, 1.0],
                   a_s=2.0, d_s=0.04)
        llp = dict(x0_var=10.0, sigma_v2=1.0, sigma_w2=0.1, a_v=2.0, b_v=1.0, a_w=2.0, b_w=1.0)
        good = []
        for model, params in (("ll_pf", llp), ("ll_pl", llp), ("sv_pf", dict(llp, sigma2=0.04)),
                              ("sv_pl", svp)):
            for n in (1, 255, 1024, 5000, 1 << 20):
                for scheme in range(4):
                    for strat in range(4):
                        for ipt in (0, 1, 2, 4, 8):
                            for prec in (0, 1):
                                for flags in (0, 1, 2, 4, 8):
                                    c = pf.make_config(model, n, 1, scheme=scheme, precision=prec,
                                                       strategy=strat, items_per_thread=ipt,
                                                       flags=flags, **params)
                                    nb = L.pf_workspace_bytes(ctypes.byref(c))
                                    L.pf_last_error()
                                    if nb:
                                        good.append(c)
        for c in good[::50]:
            h = vp()
            assert L.pf_create(ctypes.byref(c), None, 0, None, ctypes.byref(h)) != 0   # no device
            assert not h.value
            assert L.pf_create(ctypes.byref(c), vp(16), 1 << 40, None, ctypes.byref(h)) != 0
            assert L.pf_create(ctypes.byref(c), vp(4096), 1 << 40, None, ctypes.byref(h)) != 0
        for bad in (None,):
            assert L.pf_step(bad, None, 1) != 0
            assert L.pf_loglik(bad, None) != 0
            assert L.pf_moments(bad, None, 0) != 0
            assert L.pf_destroy(bad) == 0
            assert L.pf_checkpoint_bytes(bad) == 0
            assert L.pf_checkpoint_save(bad, None, 0) != 0
            assert L.pf_checkpoint_restore(bad, None, 0) != 0
            assert L.pf_debug_particles(bad, None, 0, None) != 0
            assert L.pf_timing_start(bad, 1, 1) != 0
        assert L.pf_batch_bytes(0, 8, 10) == 0 and L.pf_batch_bytes(64, 0, 0) > 0
        assert L.pf_batch_bytes(64, 8, 1 << 20) > L.pf_batch_bytes(64, 8, 0)
        assert L.pf_batch_create(None, 0, 0, 0, None) != 0
        assert L.pf_step_batch(None, 0, None) != 0
        q = vp(4096)
        assert L.pf_debug_search(None, q, 10, 1, 1, q, None) != 0
        assert L.pf_debug_search(q, None, 10, 1, 1, q, None) != 0
        assert L.pf_debug_search(q, q, 10, 1, 9, q, None) != 0
        assert L.pf_debug_search_noalloc(q, q, (1 << 20) + 1, 1, pf.SEARCH_CUTPOINT, q, None) != 0
        assert L.pf_debug_search_noalloc(q, q, 10, 1, pf.SEARCH_BINARY, q, None) == pf.EDEVICE
        y = (ctypes.c_double * 3)(0.1, 0.2, 0.3)
        c = good[0]
        ms = ctypes.c_double()
        assert L.pf_autotune(ctypes.byref(c), y, 2, None, ctypes.byref(ms)) != 0
        assert L.pf_autotune(ctypes.byref(c), y, 3, None, ctypes.byref(ms)) != 0
        print("ALL DONE")
    """, tmp_path)
