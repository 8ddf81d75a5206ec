"""include/ffst.h is a C header: a C99 program that includes it compiles with
warnings as errors, links against libffst.so and, on the CPU, gets the
documented errors back from calls on NULL handles and bad arguments."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1202_1773_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_SOURCE = r"""
#include <stdio.h>
#include <string.h>
#include "ffst.h"

int main(void) {
    ffst_plan* plan = NULL;
    ffst_batch* batch = NULL;
    ffst_options opt;
    int M[1] = {64}, N[1] = {64}, J[1] = {2};
    int failures = 0;
    memset(&opt, 0, sizeof opt);
    opt.aux_order = 11;                                   /* out of range */
    if (ffst_spectra_ex(64, 64, 2, &opt, &plan) != FFST_EINVAL || plan != NULL) failures++;
    if (strstr(ffst_last_error(), "aux_order") == NULL) failures++;
    if (ffst_spectra(320, 512, 3, &plan) != FFST_EUNSUPPORTED) failures++;
    if (ffst_forward(NULL, NULL, NULL, 1, NULL, NULL) != FFST_EBADPLAN) failures++;
    if (ffst_adjoint_complex(NULL, NULL, NULL, 1, NULL, NULL) != FFST_EBADPLAN) failures++;
    if (ffst_workspace_size(NULL, 4) != 0) failures++;
    if (ffst_batch_create(0, M, N, J, NULL, &batch) != FFST_EINVAL || batch != NULL) failures++;
    if (ffst_num_kernels() < 9 || ffst_kernel_name(0)[0] != 'k') failures++;
    ffst_destroy(NULL);
    ffst_batch_destroy(NULL);
    printf("%d\n", failures);
    return failures;
}
"""


def test_header_compiles_as_c_and_links(tmp_path):
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libffst.so is not built (run python -m paper_1202_1773_amd.build)")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(C_SOURCE)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(_lib.LIB_PATH)
    # a sanitizer build of the library takes its runtime from the preloaded
    # sanitizer library at run time, not from the link
    extra = [] if os.path.basename(_lib.LIB_PATH) == "libffst.so" else ["-Wl,--allow-shlib-undefined"]
    res = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                          str(src), "-o", str(exe), "-L", libdir, f"-l:{os.path.basename(_lib.LIB_PATH)}",
                          f"-Wl,-rpath,{libdir}", *extra],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.stdout, run.stderr)
    assert run.stdout.strip() == "0"


LAYOUT_SOURCE = r"""
#include <stddef.h>
#include <stdio.h>
#include "ffst.h"

int main(void) {
    printf("ffst_tuning %zu", sizeof(ffst_tuning));
    printf(" nparts %zu blocks_per_cu %zu col_values %zu row_block %zu fwd_nparts %zu\n",
           offsetof(ffst_tuning, nparts), offsetof(ffst_tuning, blocks_per_cu), offsetof(ffst_tuning, col_values),
           offsetof(ffst_tuning, row_block), offsetof(ffst_tuning, fwd_nparts));
    printf("ffst_options %zu", sizeof(ffst_options));
    printf(" max_scale_min %zu shearlet %zu complex_shearlets %zu aux_order %zu\n",
           offsetof(ffst_options, max_scale_min), offsetof(ffst_options, shearlet),
           offsetof(ffst_options, complex_shearlets), offsetof(ffst_options, aux_order));
    return 0;
}
"""


def test_struct_layouts_match_the_binding(tmp_path):
    # the ctypes structures of the binding must lay out like the header's
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_SOURCE)
    exe = tmp_path / "layout"
    res = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                          str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60).stdout.split("\n")
    for line, cls in zip(out, (_lib.ffst_tuning, _lib.ffst_options)):
        words = line.split()
        assert words[0] == cls.__name__ and int(words[1]) == ctypes.sizeof(cls), (line, cls)
        fields = dict(zip(words[2::2], (int(w) for w in words[3::2])))
        assert fields == {name: getattr(cls, name).offset for name, _ in cls._fields_}, (line, cls)
