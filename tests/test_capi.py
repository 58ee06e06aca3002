"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'mg5mi.h')
LIBPATH = os.path.join(ROOT, 'paper_2106_12631_amd', 'libmg5mi.so')


def declared():
    src = open(HEADER).read()
    return re.findall(r'^\s*(?:int|int64_t|const char\*)\s+(mg_\w+)\s*\(', src, re.M)


def test_header_declares_the_path():
    names = set(declared())
    assert {'mg_create', 'mg_destroy', 'mg_layout', 'mg_rng', 'mg_rambo', 'mg_sample',
            'mg_sigmakin', 'mg_sigmakin_hel', 'mg_adjoint', 'mg_count_nonfinite', 'mg_strerror',
            'mg_xsec_stats', 'mg_xsec_stats_workspace_bytes', 'mg_xsec', 'mg_unweight',
            'mg_unweight_workspace_bytes', 'mg_unweight_noalloc'} <= names


@pytest.mark.skipif(not os.path.exists(LIBPATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIBPATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing


@pytest.mark.skipif(not os.path.exists(LIBPATH), reason="library not built")
def test_strerror_without_gpu():
    L = ctypes.CDLL(LIBPATH)
    L.mg_strerror.restype = ctypes.c_char_p
    L.mg_strerror.argtypes = [ctypes.c_int]
    assert L.mg_strerror(0) == b"success"
    assert b"invalid" in L.mg_strerror(-1)
    assert L.mg_strerror(12345) == b"unknown error"


def test_generator_diagram_counts_and_colour_matrix():
    from paper_2106_12631_amd.gen.diagrams import ProcessDiagrams, colour_matrix
    counts = {p: ProcessDiagrams(p).ndiagrams for p in ('eemumu', 'ggtt', 'ggttg', 'ggttgg')}
    assert counts == {'eemumu': 2, 'ggtt': 3, 'ggttg': 16, 'ggttgg': 123}
    pd = ProcessDiagrams('ggtt')
    num, den = colour_matrix(pd.colour_basis(), 2)
    assert (num, den) == ([[16, -2], [-2, 16]], 3)
    # every diagram's colour factor lies in the T-string basis
    for p in ('ggttg', 'ggttgg'):
        pd = ProcessDiagrams(p)
        coefs = pd.jamp_coefficients()
        assert len(coefs) == len(pd.diagrams) and all(coefs)


def test_binding_constants_match_the_header():
    """The binding's flag bits and the Params struct follow include/mg5mi.h."""
    import paper_2106_12631_amd as mg
    src = open(HEADER).read()
    flags = dict((n, int(v)) for n, v in re.findall(r'#define MG_(FLAG_\w+) (\d+)', src))
    assert flags and all(getattr(mg, n) == v for n, v in flags.items())
    body = re.search(r'typedef struct \{(.*?)\} mg_params_t;', src, re.S).group(1)
    fields = re.findall(r'^\s*(double|int)\s+([\w, ]+);', body, re.M)
    names = [x.strip() for _, decl in fields for x in decl.split(',')]
    assert [f[0] for f in mg.Params._fields_] == names


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, 'paper_2106_12631_amd', 'libmg5cal.so')),
                    reason="calibration library not built")
def test_calibration_library_exports_its_entry_point():
    L = ctypes.CDLL(os.path.join(ROOT, 'paper_2106_12631_amd', 'libmg5cal.so'))
    assert hasattr(L, 'mgcal_run')
