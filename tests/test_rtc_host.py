"""Systems registered at run time, on the host (no GPU needed): registration
compiles the source with hipRTC against the library's kernel headers; data-
dependent control flow and sources that do not compile are refused with the
reason."""
import pytest

from paper_2609_02876_amd import _abi as A
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import user_systems as U


def test_register_compiles_and_names_the_system():
    sid = B.register_system("host_lorenz", U.LORENZ, 3, 3)
    assert sid >= 1000 and A.SYSTEMS["host_lorenz"] == (sid, 3, 3)
    sid2 = B.register_system("host_robertson", U.ROBERTSON, 3, 3, jacobian=True)
    assert sid2 == sid + 1


@pytest.mark.parametrize("snippet,what", [
    ("f[0] = y[0] > 0 ? y[0] : -y[0];", "'?'"),
    ("if (y[0] > T(0)) f[0] = y[0];", "'if'"),
    ("for (int i = 0; i < 3; ++i) f[i] = y[i];", "'for'"),
    ("while (false) {}", "'while'"),
    ("f[0] = T(y[0] > 0 && y[1] > 0);", "&&"),
    ("asm volatile(\"\");", "'asm'"),
    ("f[0] = __builtin_amdgcn_readfirstlane(y[0]);", "'__builtin_amdgcn_readfirstlane'"),
    ("f[0] = __shfl_xor(y[0], 1);", "'__shfl_xor'"),
    ("f[0] = y[threadIdx.x % 3];", "'threadIdx'"),
    ("atomicAdd(f, y[0]);", "'atomicAdd'"),
    ("__syncthreads();", "'__syncthreads'"),
])
def test_control_flow_is_refused(snippet, what):
    src = ("struct System { template <class T> __device__ static void rhs(const T* y, "
           "const T* p, T* f) { " + snippet + " } };")
    with pytest.raises(A.EnsembleError) as e:
        B.register_system("bad_" + str(abs(hash(snippet))), src, 3, 3)
    assert "straight-line" in str(e.value) and what in str(e.value)


def test_comments_and_strings_do_not_count():
    src = U.LORENZ.replace("struct System {", "// if for while ? && ||\n/* do switch */\nstruct System {")
    B.register_system("host_lorenz_commented", src, 3, 3)


def test_preprocessor_refused_and_compile_errors_reported():
    with pytest.raises(A.EnsembleError, match="preprocessor"):
        B.register_system("bad_pp", "#include <cmath>\n" + U.LORENZ, 3, 3)
    with pytest.raises(A.EnsembleError, match="does not compile"):
        B.register_system("bad_syntax", "struct System { this is not C++ };", 3, 3)
    with pytest.raises(A.EnsembleError, match="dim"):
        B.register_system("bad_dim", U.LORENZ, 0, 3)
    with pytest.raises(A.EnsembleError, match="dim <= 8"):
        B.register_system("bad_jac_dim", U.ROBERTSON, 9, 3, jacobian=True)
