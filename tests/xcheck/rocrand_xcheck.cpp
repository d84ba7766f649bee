// Independent cross-check for the oracle's base generators: prints words of
// rocRAND's Philox4x32-10 and MRG32k3a engines, built from rocRAND's source
// headers for the host CPU (no GPU is touched).  Test infrastructure only.
//
//   rocrand_xcheck philox SEED SUBSEQUENCE OFFSET COUNT [OFFSET2]
//   rocrand_xcheck mrg S10 S11 S12 S20 S21 S22 SEQUENCE SUBSEQUENCE OFFSET COUNT
//
// rocRAND's Philox subsequence s sets counter words 2 and 3 to (s mod 2^32,
// s / 2^32); its MRG32k3a sequence and subsequence jumps are 2^127 and 2^76
// steps.  Values are printed one per line in decimal.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

struct MrgWithState : rocrand_device::mrg32k3a_engine {
    void set_state(const unsigned int s[6])
    {
        for (int i = 0; i < 3; i++) {
            m_state.g1[i] = s[i];
            m_state.g2[i] = s[3 + i];
        }
    }
};

unsigned long long arg(const char *s) { return std::strtoull(s, nullptr, 0); }

}  // namespace

int main(int argc, char **argv)
{
    if ((argc == 6 || argc == 7) && std::strcmp(argv[1], "philox") == 0) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(arg(argv[2]), arg(argv[3]), arg(argv[4]), &st);
        if (argc == 7)                      // a second skip reaches blocks >= 2^62
            skipahead(arg(argv[6]), &st);
        unsigned long long count = arg(argv[5]);
        for (unsigned long long i = 0; i < count; i++)
            std::printf("%u\n", rocrand(&st));
        return 0;
    }
    if (argc == 12 && std::strcmp(argv[1], "mrg") == 0) {
        unsigned int s[6];
        for (int i = 0; i < 6; i++)
            s[i] = static_cast<unsigned int>(arg(argv[2 + i]));
        MrgWithState g;
        g.set_state(s);
        g.discard_sequence(arg(argv[8]));
        g.discard_subsequence(arg(argv[9]));
        g.discard(arg(argv[10]));
        unsigned long long count = arg(argv[11]);
        for (unsigned long long i = 0; i < count; i++)
            std::printf("%u\n", g.next());
        return 0;
    }
    std::fprintf(stderr, "usage: see source\n");
    return 2;
}
