"""Admission policy of the solve server (host-only C++ in
paper_2602_05686_amd/csrc/admission.h), driven by a small g++ program:
FIFO order without overtaking, the byte budget and the slot cap, shrinking
reservations after setup, and the setup-peak estimate's monotonicity; the
driver is built with AddressSanitizer and UndefinedBehaviorSanitizer."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_05686_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "admission.h"
using namespace matamg;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
static bool same(const std::vector<uint64_t>& a, std::initializer_list<uint64_t> b) {
    return a == std::vector<uint64_t>(b);
}
int main() {
    {   // budget binds: head waits, later small requests do not overtake it
        Admission a(100, 8);
        CHECK(a.fits_ever(100) && !a.fits_ever(101));
        a.push(1, 60); a.push(2, 50); a.push(3, 10);
        CHECK(same(a.admit(), {1}));
        CHECK(a.used() == 60 && a.waiting() == 2 && a.active() == 1);
        CHECK(a.admit().empty());            // 2 does not fit; 3 may not overtake
        a.resize(1, 20);                     // setup done: only the resident bytes stay reserved
        CHECK(same(a.admit(), {2, 3}));
        CHECK(a.used() == 80 && a.peak_used() == 80);
        a.release(2);
        CHECK(a.used() == 30 && a.active() == 2);
        a.release(2);                        // releasing twice is harmless
        CHECK(a.used() == 30);
    }
    {   // slot cap binds
        Admission a(1000, 2);
        for (uint64_t i = 1; i <= 5; ++i) a.push(i, 1);
        CHECK(same(a.admit(), {1, 2}));
        CHECK(a.admit().empty());
        a.release(1);
        CHECK(same(a.admit(), {3}));
        a.release(2); a.release(3);
        CHECK(same(a.admit(), {4, 5}));
        CHECK(a.waiting() == 0 && a.active() == 2);
    }
    {   // peak tracks growth through resize
        Admission a(100, 4);
        a.push(1, 10);
        a.admit();
        a.resize(1, 70);
        CHECK(a.peak_used() == 70 && a.used() == 70);
    }
    {   // estimate grows with every size and covers the dense coarse solve
        int64_t e0 = estimate_setup_bytes(1000, 27000, 900, 8, 3, 5000);
        CHECK(e0 > 16 * 1000 * 1000);
        CHECK(estimate_setup_bytes(2000, 27000, 900, 8, 3, 5000) > e0);
        CHECK(estimate_setup_bytes(1000, 54000, 900, 8, 3, 5000) > e0);
        CHECK(estimate_setup_bytes(1000, 27000, 1800, 8, 3, 5000) > e0);
        // the dense term saturates at max_coarse
        int64_t big = estimate_setup_bytes(100000, 2700000, 97336, 8, 3, 5000);
        int64_t bigger = estimate_setup_bytes(200000, 2700000, 97336, 8, 3, 5000);
        CHECK(bigger - big < 2 * 16 * (int64_t)5000 * 5000);
    }
    std::printf("OK\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("adm")
    src = d / "adm.cpp"
    src.write_text(DRIVER)
    exe = d / "adm"
    # host code under AddressSanitizer and UndefinedBehaviorSanitizer (no
    # recovery) where the runtime is installed
    libasan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
           if os.path.isabs(libasan) and os.path.exists(libasan) else [])
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", *san, "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return exe


def test_admission_policy(driver):
    res = subprocess.run([str(driver)], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "OK", res.stdout + res.stderr
