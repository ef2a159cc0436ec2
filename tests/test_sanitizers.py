"""Host-side sanitizer run (CPU only): the library's translation units are
rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer on the host
side, and a C driver built with the same sanitizers exercises every
argument-error path and the injected-failure path of the C ABI (no GPU call
is made).  Any sanitizer report makes the driver exit non-zero."""
import concurrent.futures as cf
import os
import subprocess
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_03983_amd", "csrc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

DRIVER = textwrap.dedent(r"""
    #include <stdio.h>
    #include <stdlib.h>
    #include "apsp.h"
    #define EXPECT(cond) do { if (!(cond)) { printf("FAIL line %d\n", __LINE__); return 1; } } while (0)
    int main(void) {
        apsp_opts_t o = {0};
        void *fake = (void *)0x1000;
        int64_t v;
        EXPECT(apsp_fw(NULL, 7, 4, fake, 4, &o, NULL) == APSP_E_ARG);
        EXPECT(apsp_rkleene(NULL, APSP_I32, -1, fake, 4, &o, NULL) == APSP_E_ARG);
        EXPECT(apsp_square(NULL, APSP_F32, 8, fake, 4, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_solve(NULL, APSP_I32, 8, NULL, 8, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_closure(NULL, APSP_I32, 8, fake, 8, NULL, NULL) == APSP_E_ARG);
        o.block = 96;
        EXPECT(apsp_fw(NULL, APSP_I32, 8, fake, 8, &o, NULL) == APSP_E_ARG);
        o.block = 0;
        EXPECT(minplus_gemm(NULL, APSP_I32, 4, 4, 4, fake, 4, fake, 4, fake, 4, NULL, NULL) == APSP_E_ARG);
        EXPECT(minplus_gemm(NULL, APSP_I32, 2, 2, 2, fake, 1, fake, 2, fake, 2, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_validate(NULL, APSP_I32, 4, fake, 4, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_validate(NULL, APSP_I32, 4, fake, 4, NULL, &v) == APSP_E_ARG);
        EXPECT(apsp_predecessors(NULL, APSP_I32, 4, fake, 4, fake, 4, (int32_t *)fake, 4, NULL) == APSP_E_ARG);
        int32_t sizes[2] = {3, 9000};
        EXPECT(apsp_batched(NULL, APSP_I32, 2, fake, fake, fake, sizes, NULL, NULL) == APSP_E_UNSUPPORTED);
        EXPECT(apsp_batched(NULL, APSP_I32, -1, fake, fake, fake, sizes, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_plan(NULL, APSP_I32, 100, 0.1, 1, 1, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_plan(NULL, (apsp_dtype_t)9, 100, 0.1, 1, 1, NULL, NULL) == APSP_E_ARG);
        EXPECT(apsp_candidate(-1, &o) == APSP_E_ARG);
        for (int i = 0; i < apsp_candidate_count(); ++i) EXPECT(apsp_candidate(i, &o) == APSP_OK);
        EXPECT(apsp_costmodel_init(NULL, 0, 1) == APSP_E_ARG);
        apsp_ctx_t *c = NULL;
        EXPECT(apsp_create(NULL, 0) == APSP_E_ARG);
        EXPECT(apsp_create(&c, -3) == APSP_E_ARG);
        EXPECT(apsp_create(&c, 0) == APSP_E_HIP);   /* APSP_FAULT=create in the environment */
        EXPECT(c == NULL);
        EXPECT(apsp_destroy(NULL) == APSP_OK);
        EXPECT(apsp_last_error()[0] != 0);
        printf("sanitized host paths ok\n");
        return 0;
    }
""")


def _compile(args):
    src, obj = args
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return obj


def test_host_paths_under_asan_and_ubsan(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    jobs = [(s, str(tmp_path / (os.path.basename(s) + ".o"))) for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = list(ex.map(_compile, jobs))
    lib = str(tmp_path / "libapsp_san.so")
    subprocess.run(["/opt/rocm/bin/hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *HOST_SAN, "-o", lib, *objs],
                   check=True, capture_output=True, text=True)
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = str(tmp_path / "driver")
    subprocess.run(["clang", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g",
                    "-I", os.path.join(ROOT, "include"), str(drv), lib, f"-Wl,-rpath,{tmp_path}",
                    "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True, capture_output=True, text=True, env=dict(os.environ, PATH="/opt/rocm/llvm/bin:" + os.environ["PATH"]))
    env = dict(os.environ, APSP_FAULT="create", ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "sanitized host paths ok" in out.stdout
