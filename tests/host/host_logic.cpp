// The host-side planning of libfdtd, run without a GPU.  This program compiles
// the library's host source on its own (the kernel entry points stay unresolved:
// nothing here launches a kernel or touches a device) and prints what the
// library would hand to the device, for the CPU tests to check:
//
//   host_logic worklist NX NY NZ TX ROWS SLOTS
//       the work list of one launch over the board's whole tiles of TX columns and
//       ROWS owned rows, dealt to 8 XCDs of SLOTS concurrent blocks each: one line
//       "board tx ty kb ke" per entry (board -1: an idle entry)
//   host_logic coefs NX NY NZ DX DY DZ NLX NHX NLY NHY NLZ NHZ M R KMAX DT AXIS
//       the FP32 coefficient table of one axis (Eq. 5 grading): one line per
//       coefficient kind and half (node, half node), NAXIS + 1 values each
//   host_logic matsplit NX NY NZ FILE
//       a material board's split between the plain two-step kernel and its
//       material variants, from FILE: one byte per node, x fastest, bit 1 where
//       the node's PML coefficients are rebuilt, bit 2 where an edge conducts;
//       "split S mat_ty T" then one line "rb|cd|plain tx ty kb ke" per piece
//   host_logic plan TX TY PER CUS SPEC
//       one round of a batched call (fdtd_step_many) in the lead's shape
//       TX x TY x PER on a device of CUS compute units (occupancy 1), for the
//       boards of SPEC, one a line: "NX NY NZ STEPS MAT WIDE NEEDFILE" (MAT 1: a
//       material board split by NEEDFILE as for matsplit; "-": none).  Prints
//       "order h..." (boards in launch order), per span "span W STEPS S0 S1 TAIL",
//       per list of the span "list KIND" and one line "e b tx ty kb ke" per entry,
//       "node_tail H REL FLIP" per material board's single step, and
//       "adv B STEPS LAUNCHES" per board of the order
#include "fdtd_host.cpp"

#include <cstdlib>
#include <fstream>
#include <memory>
#include <sstream>

// The kernels' occupancy is a property of the device; the plans here are built
// for one block per compute unit of every shape.
namespace fdtd {
int field_step_occupancy(int, int, bool) { return 1; }
int field_step2_occupancy(int, bool) { return 1; }
int field_step2_material_occupancy(int, int, bool) { return 1; }
}  // namespace fdtd

static bool read_need(const char* path, int nx, int ny, int nz, std::vector<uint8_t>& tile_need)
{
    const size_t plane = (size_t)(nx + 1) * (ny + 1);
    std::vector<uint8_t> need(plane * (nz + 1));
    FILE* f = fopen(path, "rb");
    if (!f) return false;
    const bool ok = fread(need.data(), 1, need.size(), f) == need.size();
    fclose(f);
    if (!ok) return false;
    // as the class build does: plane by plane, each kind of need on its own
    int hcx = 0, hcy = 0;
    tile_counts(nx, ny, 64, owned_rows(fdtd::kHybridTY, 2), &hcx, &hcy);
    tile_need.clear();
    std::vector<int32_t> pre;
    for (int k = 0; k <= nz; ++k) {
        uint8_t bits = 0;
        for (size_t n = 0; n < plane; ++n) bits |= need[k * plane + n];
        if (!bits) continue;
        if (tile_need.empty()) tile_need.assign((size_t)hcx * hcy * (nz + 1), 0);
        for (uint8_t bit = 1; bit <= 2; bit <<= 1)
            if (bits & bit) mark_tile_need(&need[k * plane], nx, ny, bit, pre, &tile_need[k], nz + 1);
    }
    return true;
}

int main(int argc, char** argv)
{
    using namespace fdtd;
    if (argc >= 8 && !strcmp(argv[1], "worklist")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
        const int tx = atoi(argv[5]), rows = atoi(argv[6]), slots = atoi(argv[7]);
        std::vector<TileRef> whole, out;
        board_tiles(0, nx, ny, nz, tx, rows, whole);
        build_work(whole, slots, out);
        for (const TileRef& t : out) printf("%d %d %d %d %d\n", t.board, t.tx, t.ty, t.kb, t.ke);
        return 0;
    }
    if (argc >= 19 && !strcmp(argv[1], "coefs")) {
        fdtd_grid_desc d{};
        d.nx = atoi(argv[2]);
        d.ny = atoi(argv[3]);
        d.nz = atoi(argv[4]);
        d.dx = atof(argv[5]);
        d.dy = atof(argv[6]);
        d.dz = atof(argv[7]);
        for (int q = 0; q < 6; ++q) d.npml[q] = atoi(argv[8 + q]);
        d.pml_m = atof(argv[14]);
        d.pml_R = atof(argv[15]);
        d.pml_kappa_max = atof(argv[16]);
        const double dt = atof(argv[17]);
        const int axis = atoi(argv[18]);
        const int n = axis == 0 ? d.nx : axis == 1 ? d.ny : d.nz;
        const std::vector<float> t = coef_table(d, axis, dt);
        for (int row = 0; row < kNumCoef * 2; ++row) {
            for (int i = 0; i <= n; ++i) printf("%.9g ", (double)t[(size_t)row * (n + 1) + i]);
            printf("\n");
        }
        return 0;
    }
    if (argc >= 6 && !strcmp(argv[1], "matsplit")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
        std::vector<uint8_t> tile_need;
        if (!read_need(argv[5], nx, ny, nz, tile_need)) return 3;
        MaterialSplit ms;
        split_material(nx, ny, nz, tile_need, ms);
        printf("split %d mat_ty %d\n", ms.split, ms.mat_ty);
        for (const TileRef& t : ms.rb) printf("rb %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        for (const TileRef& t : ms.cd) printf("cd %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        for (const TileRef& t : ms.plain) printf("plain %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        return 0;
    }
    if (argc >= 7 && !strcmp(argv[1], "plan")) {
        std::vector<std::unique_ptr<fdtd_grid>> hs;
        std::vector<int64_t> n;
        std::ifstream spec(argv[6]);
        std::string line;
        while (std::getline(spec, line)) {
            std::istringstream in(line);
            int nx, ny, nz, mat, wide;
            int64_t steps;
            std::string needfile;
            if (!(in >> nx >> ny >> nz >> steps >> mat >> wide >> needfile)) continue;
            auto g = std::make_unique<fdtd_grid>();
            g->d.nx = nx;
            g->d.ny = ny;
            g->d.nz = nz;
            g->wide = wide != 0;
            g->mat = mat != 0;
            g->cus = atoi(argv[5]);
            g->tile_x = atoi(argv[2]);
            g->tile_y = atoi(argv[3]);
            g->tile_steps = atoi(argv[4]);
            if (g->mat) {
                std::vector<uint8_t> tile_need;
                if (needfile != "-" && !read_need(needfile.c_str(), nx, ny, nz, tile_need)) return 3;
                MaterialSplit ms;
                split_material(nx, ny, nz, tile_need, ms);
                g->mat_ty = ms.mat_ty;
                g->pc_plain = ms.plain;
                g->pc_cd = ms.cd;
                g->pc_rb = ms.rb;
            }
            hs.push_back(std::move(g));
            n.push_back(steps);
        }
        std::vector<fdtd_grid*> gs;
        for (auto& g : hs) gs.push_back(g.get());
        RoundHost r;
        plan_round(gs.data(), (int)gs.size(), n.data(), r);
        printf("order");
        for (int h : r.order) printf(" %d", h);
        printf("\n");
        for (const Span& sp : r.spans) {
            printf("span %d %d %lld %lld %d\n", sp.w, sp.steps, (long long)sp.s0, (long long)sp.s1, (int)sp.tail);
            for (int l = 0; l < sp.nl; ++l) {
                printf("list %d\n", sp.kind[l]);
                for (int q = 0; q < sp.count[l]; ++q) {
                    const TileRef& t = r.items[(size_t)sp.off[l] + q];
                    printf("e %d %d %d %d %d\n", t.board, t.tx, t.ty, t.kb, t.ke);
                }
            }
        }
        for (const NodeTail& t : r.node_tails) printf("node_tail %d %d %d\n", t.h, t.rel, t.flip);
        for (size_t b = 0; b < gs.size(); ++b)
            printf("adv %zu %lld %lld\n", b, (long long)r.adv[2 * b], (long long)r.adv[2 * b + 1]);
        return 0;
    }
    fprintf(stderr, "usage: host_logic worklist ... | coefs ... | matsplit ... | plan ...\n");
    return 2;
}
